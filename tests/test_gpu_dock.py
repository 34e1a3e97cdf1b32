"""GPU parity of the docking search (Lamarckian GA + ADADELTA) with the oracle.

The search is stochastic and chaotic (a tournament between two close
energies can go either way in FP32 vs FP64), so parity is checked where it
is well defined: identical random streams (the initial population), every
returned pose re-scores to its energy, exact evaluation accounting,
per-ligand reproducibility from (seed, ligand id), and the distribution of
best energies over independent seeds (Mann-Whitney U, medians within
0.3 kcal/mol).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

E_ABS, E_REL = 1e-3, 1e-5


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03678_amd as pkg
    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def setup(pkg, ff, orc):
    rec = synth.receptor(31, 1200, side=16.0)
    grid = synth.make_grid(32, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    ctx = pkg.create(ff, 0)
    ctx.ad_load_grids(grid, G.values())
    yield ctx, grid, G
    ctx.close()


def test_initial_population_matches_oracle_streams(pkg, setup, orc):
    ctx, grid, G = setup
    lig = synth.ligand(40, 30, 7)
    batch = ctx.ad_load_ligands([lig])
    L = orc.ligand(lig)
    seed = (123 << 32) | 456
    gp = ctx.ad_initial_population(batch, 0, 77, 3, 200, seed)
    for i in range(200):
        go = orc.init_individual(L, G, seed, 77, 3, i)
        assert np.allclose(gp[i], go.astype(np.float32), rtol=0, atol=2e-6), i
    batch.free()


def test_local_search_improves_and_rescores(pkg, setup, orc):
    ctx, grid, G = setup
    ligs = [synth.ligand(41 + i, n, t) for i, (n, t) in enumerate([(18, 4), (35, 9), (70, 20)])]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    n = 96
    idx = (np.arange(n) % 3).astype(np.int32)
    ntor = np.array([OL[i].n_tor for i in idx])
    g0 = synth.random_genotypes(5, n, ntor, grid, margin=3.0, normalize_q=True)
    E0, _, _ = ctx.ad_score_poses(batch, idx, g0)
    p = pkg.make_params()
    g1, E1 = ctx.ad_local_search(batch, idx, g0, p, 100)
    assert np.all(E1 <= E0)
    # the returned pose re-scores to the returned energy (GPU and oracle)
    E1r, _, _ = ctx.ad_score_poses(batch, idx, g1)
    assert np.array_equal(E1r, E1)
    Eo, _, _ = orc.score_batch(OL, idx, G, g1)
    assert np.all(np.abs(E1 - Eo) <= np.maximum(E_ABS, E_REL * np.abs(Eo)))
    # statistically as good as the FP64 oracle's ADADELTA from the same starts
    Eorc = np.array([orc.adadelta(OL[i], G, oracle.make_params(), g0[k].astype(np.float64), 100)[1]
                     for k, i in enumerate(idx)])
    assert abs(np.median(E1) - np.median(Eorc)) < 0.15 * abs(np.median(Eorc)) + 0.5
    batch.free()


def test_local_search_first_iterations_follow_oracle(pkg, setup, orc):
    """One and three ADADELTA evaluations from the same start: the GPU keeps the
    same best pose as the FP64 oracle (the trajectories only drift apart by
    rounding later)."""
    ctx, grid, G = setup
    lig = synth.ligand(45, 25, 6)
    batch = ctx.ad_load_ligands([lig])
    L = orc.ligand(lig)
    g0 = synth.random_genotypes(6, 32, L.n_tor, grid, margin=3.0, normalize_q=True)
    p = pkg.make_params()
    for iters in (1, 3):
        g1, E1 = ctx.ad_local_search(batch, np.zeros(32, np.int32), g0, p, iters)
        for k in range(32):
            bo, Eo = orc.adadelta(L, G, oracle.make_params(), g0[k].astype(np.float64), iters)
            assert abs(E1[k] - Eo) <= max(1e-2, 1e-4 * abs(Eo)), (iters, k, E1[k], Eo)
            assert np.allclose(g1[k][:3], bo[:3], atol=1e-3)
    batch.free()


def chain_ligand(n, n_rot):
    """Zigzag carbon chain (1.5 A bonds, 109.5 degree angles) whose bonds 1 ..
    n_rot are rotatable; alternating charges summing to zero."""
    half = np.deg2rad(109.5) / 2
    x = np.zeros((n, 3))
    for i in range(1, n):
        x[i] = x[i - 1] + 1.5 * np.array([np.sin(half), np.cos(half) * (1 if i % 2 else -1), 0.0])
    x -= x.mean(0)
    q = np.where(np.arange(n) % 2 == 0, 0.1, -0.1)
    q -= q.mean()
    rot = np.zeros(n - 1, np.uint8)
    rot[1:1 + n_rot] = 1
    return synth.Ligand(np.full(n, synth.TYPE_ID["C"], np.int32), q.astype(np.float32), x.astype(np.float32),
                        np.array([[i, i + 1] for i in range(n - 1)], np.int32), rot)


def small_params(pkg, **kw):
    d = dict(nrun=4, pop=30, max_gens=8, ls_rate=0.1, ls_iters=40)
    d.update(kw)
    return pkg.make_params(**d)


def test_dock_accounting_rescoring_and_reproducibility(pkg, setup, orc):
    ctx, grid, G = setup
    ligs = [synth.ligand(50 + i, n, t) for i, (n, t) in enumerate([(12, 2), (26, 6), (44, 12), (66, 18)])]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    p = small_params(pkg)
    seed = 2024
    r = ctx.ad_dock_batch(batch, p, seed, per_run=True)
    n_ls = 3
    per_gen = (30 - 1) + n_ls * 40
    assert np.all(r["generations"] == 8)
    assert np.all(r["evals"] == 4 * (30 + 8 * per_gen))
    # every returned pose re-scores to its energy; the best is the min over runs
    for l in range(4):
        assert r["best_energy"][l] == r["run_energy"][l].min()
        assert r["best_run"][l] == int(np.argmin(r["run_energy"][l]))
        Eo, _, To = orc.score(OL[l], G, r["best_genotype"][l].astype(np.float64))
        assert abs(r["best_energy"][l] - Eo) <= max(E_ABS, E_REL * abs(Eo))
        assert abs(r["best_score"][l] - To[2]) <= max(E_ABS, E_REL * abs(To[2]))
        Er, _, _ = ctx.ad_score_poses(batch, np.full(4, l, np.int32), r["run_genotype"][l])
        assert np.array_equal(Er, r["run_energy"][l])
    # deterministic, and a ligand's result depends only on (seed, its id)
    r2 = ctx.ad_dock_batch(batch, p, seed, per_run=True)
    assert np.array_equal(r["run_energy"], r2["run_energy"])
    assert np.array_equal(r["run_genotype"], r2["run_genotype"])
    solo = ctx.ad_load_ligands([ligs[2]])
    r3 = ctx.ad_dock_batch(solo, p, seed, lig_ids=np.array([2], np.uint32), per_run=True)
    assert np.array_equal(r3["run_energy"][0], r["run_energy"][2])
    # docking a subset of the batch (the screened path) gives the same results
    r5 = ctx.ad_dock_select(batch, np.array([2, 0], np.int32), p, seed, per_run=True)
    assert np.array_equal(r5["run_energy"], r["run_energy"][[2, 0]])
    assert np.array_equal(r5["best_genotype"], r["best_genotype"][[2, 0]])
    assert np.array_equal(r5["best_score"], r["best_score"][[2, 0]])
    assert np.all(r5["evals"] == r["evals"][[2, 0]])
    with pytest.raises(pkg.AddockError):
        ctx.ad_dock_select(batch, np.array([4], np.int32), p, seed)
    assert len(ctx.ad_dock_select(batch, np.zeros(0, np.int32), p, seed)["best_energy"]) == 0
    r4 = ctx.ad_dock_batch(batch, p, seed + 1, per_run=True)
    assert not np.array_equal(r4["run_energy"], r["run_energy"])
    # the search improves on the initial population
    init = np.array([[ctx.ad_score_poses(batch, np.full(30, l, np.int32),
                                         ctx.ad_initial_population(batch, l, l, run, 30, seed))[0].min()
                      for run in range(4)] for l in range(4)])
    assert np.all(r["run_energy"] <= init)
    assert np.mean(r["run_energy"] < init - 1.0) > 0.5
    solo.free()
    batch.free()


def test_schedules_give_identical_results(pkg, setup):
    """Both atom-capacity buckets, eager and graph replay, forced and
    autotuned LDS pair staging, every local-search launch shape (pair-loop
    unroll 1 and 2, fewer work-groups per CU) forced and autotuned: bitwise
    the same docking results."""
    ctx, grid, G = setup
    # sizes across both buckets and the packing limit; large pair lists make
    # lanes of different steps add to the same atoms (where an order change
    # between schedules would show in the last bits).  The pair-step counts
    # cover one step, odd and even counts, and last steps from 1 to 62 live
    # lanes, on 32-lane halves (packed) and whole wavefronts
    sizes = [(12, 2), (30, 7), (70, 20), (50, 12), (90, 25), (20, 5), (40, 10), (60, 16), (64, 24), (100, 30),
             (33, 8), (45, 13), (128, 32), (58, 14), (28, 7)]
    ligs = [synth.ligand(70 + i, n, t) for i, (n, t) in enumerate(sizes)]
    batch = ctx.ad_load_ligands(ligs)
    p = small_params(pkg, ls_iters=30, max_gens=5)
    ref = None
    try:
        for use_graph, autotune, stage in [(False, False, 0), (True, False, 0), (False, False, 2048),
                                           (True, False, 256), (True, True, -1), (True, True, -1)]:
            ctx.ad_set_schedule(use_graph, autotune, stage)
            r = ctx.ad_dock_batch(batch, p, 77, per_run=True)
            info = ctx.ad_get_schedule()
            assert info["graph"] == use_graph
            assert info["stage_pairs"][0] >= 0 and info["stage_pairs"][1] >= 0   # both buckets used
            if stage == 0:
                assert info["stage_pairs"] == [0, 0]
            if ref is None:
                ref = r
                continue
            for k in ("run_energy", "run_genotype", "evals", "best_score"):
                assert np.array_equal(r[k], ref[k]), (use_graph, autotune, stage, k)
        for unroll, wgcu, autotune in [(2, 0, False), (1, 8, False), (2, 12, False), (0, 0, True), (0, 0, True)]:
            ctx.ad_set_schedule(True, autotune, -1 if autotune else 0)
            ctx.ad_set_launch_shape(unroll, wgcu)
            r = ctx.ad_dock_batch(batch, p, 77, per_run=True)
            shape = ctx.ad_get_launch_shape()
            # forced: both buckets take it; tuned: each bucket picks its own
            assert set(shape["unroll"]) <= {1, 2} and (not unroll or shape["unroll"] == [unroll] * 2), shape
            assert all(1 <= w <= (wgcu or 16) for w in shape["wg_per_cu"]), shape
            for k in ("run_energy", "run_genotype", "evals", "best_score"):
                assert np.array_equal(r[k], ref[k]), (unroll, wgcu, autotune, shape, k)
        ctx.ad_set_launch_shape(0, 0)
        # the persistent work queue (GA and local search), with other shapes
        # and staging, eager and as a graph
        for unroll, wgcu, stage, use_graph in [(1, 0, 0, True), (2, 8, 0, True), (1, 0, 256, False), (2, 0, 0, False)]:
            ctx.ad_set_schedule(use_graph, False, stage)
            ctx.ad_set_launch_shape(unroll, wgcu)
            ctx.ad_set_work_queue(1)
            r = ctx.ad_dock_batch(batch, p, 77, per_run=True)
            assert ctx.ad_get_work_queue() == [1, 1]
            assert ctx.ad_get_schedule()["graph"] == use_graph
            for k in ("run_energy", "run_genotype", "evals", "best_score"):
                assert np.array_equal(r[k], ref[k]), ("queue", unroll, wgcu, stage, use_graph, k)
        ctx.ad_set_work_queue(0)
        ctx.ad_set_schedule()
        ctx.ad_set_launch_shape(0, 0)
        r = ctx.ad_dock_batch(batch, p, 77, per_run=True)
        assert ctx.ad_get_work_queue() == [0, 0]
        assert np.array_equal(r["run_energy"], ref["run_energy"])
        ctx.ad_set_work_queue(-1)
        # chains of launches: each bucket's runs in parts on their own
        # streams, with and without the queue, graph and eager with timing
        for parts, queue, timing in [(1, 0, False), (3, 1, False), (4, 0, False), (2, 0, True), (3, 0, True)]:
            ctx.ad_set_chains(parts)
            ctx.ad_set_work_queue(queue)
            ctx.ad_set_kernel_timing(timing)
            r = ctx.ad_dock_batch(batch, p, 77, per_run=True)
            ctx.ad_set_kernel_timing(False)
            assert ctx.ad_get_chains()[0] == parts and 1 <= ctx.ad_get_chains()[1] <= parts
            assert ctx.ad_get_schedule()["graph"] == (not timing)
            for k in ("run_energy", "run_genotype", "evals", "best_score"):
                assert np.array_equal(r[k], ref[k]), ("chains", parts, queue, timing, k)
        ctx.ad_set_chains(2)
        ctx.ad_set_work_queue(-1)
        # kernel timing runs the loop eagerly, with the same results
        ctx.ad_set_kernel_timing(True)
        r = ctx.ad_dock_batch(batch, p, 77, per_run=True)
        ctx.ad_set_kernel_timing(False)
        assert not ctx.ad_get_schedule()["graph"]
        assert np.array_equal(r["run_energy"], ref["run_energy"])
        # a subset that holds only the small bucket
        r2 = ctx.ad_dock_select(batch, np.array([3, 0, 13], np.int32), p, 77, per_run=True)
        assert ctx.ad_get_schedule()["stage_pairs"][1] == -1
        assert np.array_equal(r2["run_energy"], ref["run_energy"][[3, 0, 13]])
    finally:
        ctx.ad_set_schedule()
        ctx.ad_set_launch_shape(0, 0)
        ctx.ad_set_work_queue(-1)
        ctx.ad_set_chains(2)
        batch.free()


def test_work_queue_with_stopping_runs(pkg, setup):
    """Runs that stop on their own (autostop; Solis-Wets) with the
    persistent work queue: items of stopped runs are skipped, packed
    work-groups whose two halves have both stopped end at once, and every
    result is bitwise the one without the queue.  Such calls keep one chain
    of launches per bucket whatever ad_set_chains asks."""
    ctx, grid, G = setup
    spec = [(10, 1), (16, 3), (24, 6), (32, 9), (40, 10), (70, 18), (20, 4), (55, 12)]
    ligs = [synth.ligand(300 + i, n, t) for i, (n, t) in enumerate(spec)]
    batch = ctx.ad_load_ligands(ligs)
    cases = [small_params(pkg, nrun=5, max_gens=150, max_evals=10**9, ls_iters=30, autostop=1),
             small_params(pkg, nrun=4, max_gens=12, ls_method=1, autostop=1)]
    try:
        for i, p in enumerate(cases):
            out = []
            for mode, parts in ((0, 1), (1, 1), (1, 2), (0, 3)):
                ctx.ad_set_work_queue(mode)
                ctx.ad_set_chains(parts)
                out.append(ctx.ad_dock_batch(batch, p, 31, per_run=True))
                assert ctx.ad_get_work_queue() == [mode, mode], (i, mode)
                assert ctx.ad_get_chains() == [1, 1]   # stopping runs: one part per bucket
            if i == 0:
                assert (out[0]["generations"] < 150).any()   # some runs stopped
            for o in out[1:]:
                for k in ("run_energy", "run_genotype", "evals", "best_score", "generations"):
                    assert np.array_equal(out[0][k], o[k]), (i, k)
    finally:
        ctx.ad_set_work_queue(-1)
        ctx.ad_set_chains(2)
        batch.free()


def test_packed_local_search_follows_the_unpacked_one(pkg, setup, orc):
    """Ligands of at most 32 atoms and 25 torsions run their ADADELTA search
    two individuals per wavefront.  The packed evaluation only sums in
    another order (one wavefront half), so short searches follow the
    unpacked ones bitwise unless an FP32 rounding flips; evaluation counts
    are identical and every returned pose re-scores exactly.  nrun * n_ls is
    odd (5 x 3), so the last work-group of every ligand has an idle half."""
    ctx, grid, G = setup
    spec = [(8, 1), (16, 3), (24, 6), (32, 9), (40, 10), (30, 25), (20, 4)]
    ligs = [synth.ligand(120 + i, n, t) for i, (n, t) in enumerate(spec)]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    small = [l.n_atoms <= 32 and OL[i].n_tor <= 25 for i, l in enumerate(ligs)]
    p = small_params(pkg, nrun=5, max_gens=4, ls_iters=30)
    try:
        ctx.ad_set_schedule(pack_small=True)
        r1 = ctx.ad_dock_batch(batch, p, 9, per_run=True)
        assert ctx.ad_get_schedule()["packed_runs"] == 5 * sum(small)
        ctx.ad_set_schedule(pack_small=False)
        r0 = ctx.ad_dock_batch(batch, p, 9, per_run=True)
        assert ctx.ad_get_schedule()["packed_runs"] == 0
        # autostop (runs stop on their own) with packing
        ctx.ad_set_schedule(pack_small=True)
        ra = ctx.ad_dock_batch(batch, small_params(pkg, nrun=5, max_gens=60, ls_iters=30, autostop=1), 9,
                               per_run=True)
    finally:
        ctx.ad_set_schedule()
    assert np.array_equal(r1["evals"], r0["evals"])
    same = np.mean(r1["run_energy"] == r0["run_energy"])
    assert same >= 0.9, same
    assert np.array_equal(r1["run_energy"][~np.array(small)], r0["run_energy"][~np.array(small)])
    for r in (r1, ra):
        for l in range(len(ligs)):
            Er, _, _ = ctx.ad_score_poses(batch, np.full(5, l, np.int32), r["run_genotype"][l])
            assert np.array_equal(Er, r["run_energy"][l])
            Eo, _, _ = orc.score(OL[l], G, r["best_genotype"][l].astype(np.float64))
            assert abs(r["best_energy"][l] - Eo) <= max(E_ABS, E_REL * abs(Eo))
    per_gen = 29 + 3 * 30
    assert np.all(ra["evals"] >= 5 * (30 + 9 * per_gen)) and np.all(ra["evals"] <= 5 * (30 + 60 * per_gen))
    assert np.all((ra["evals"] - 5 * 30) % per_gen == 0)
    batch.free()


def test_packed_loading_docks_the_same(pkg, setup):
    """Ligands loaded back to back (ad_load_ligands_packed) prepare and dock
    bitwise as the same ligands loaded one structure each."""
    ctx, grid, G = setup
    pack = synth.ligand_set_fast(31, 6, atoms=(10, 90), torsions=(0, 24), packed=True)
    a = ctx.ad_load_ligands(pack.ligands())
    b = ctx.ad_load_ligands_packed(pack)
    try:
        assert a.n == b.n == 6
        for i in range(6):
            assert a.info(i) == b.info(i)
        p = small_params(pkg, ls_iters=20, max_gens=3)
        ra, rb = (ctx.ad_dock_batch(x, p, 5, per_run=True) for x in (a, b))
        for k in ("run_energy", "run_genotype", "evals"):
            assert np.array_equal(ra[k], rb[k]), k
    finally:
        a.free()
        b.free()
    with pytest.raises(pkg.AddockError):
        bad = synth.pack_ligands(pack.ligands([0, 1]))
        bad.n_atoms_per_ligand[1] = 0
        ctx.ad_load_ligands_packed(bad)


def test_streamed_docking_equals_one_batch(pkg, setup):
    """ad_dock_stream docks a back-to-back set in batches, preparing the next
    batch on a host thread while the current one docks.  Ligand i keeps
    random-stream id id0 + i, so every ligand's result equals its result in
    one batch, whatever the batch size, and a run resumed at a later ligand
    reproduces the uninterrupted one; a bad ligand stops the call and is
    named."""
    ctx, grid, G = setup
    pack = synth.ligand_set_fast(41, 11, atoms=(10, 90), torsions=(0, 24), packed=True)
    p = small_params(pkg, nrun=3, max_gens=3, ls_iters=20)
    batch = ctx.ad_load_ligands_packed(pack)
    ref = ctx.ad_dock_batch(batch, p, 17)
    batch.free()
    for bs in (4, 11, 20):
        r = ctx.ad_dock_stream(pack, bs, p, 17)
        for k in ("best_energy", "best_genotype", "best_score", "evals", "best_run", "generations"):
            assert np.array_equal(r[k], ref[k]), (bs, k)
        st = r["stats"]
        assert st["prep_s"] > 0 and st["dock_s"] > 0 and st["wall_s"] >= st["dock_s"]
    # resumed at ligand 5 (ids from 5): the same results as the uninterrupted run
    r5 = ctx.ad_dock_stream(pack.subset(list(range(5, 11))), 4, p, 17, id0=5)
    for k in ("best_energy", "best_genotype", "evals"):
        assert np.array_equal(r5[k], ref[k][5:]), k
    bad = synth.pack_ligands(pack.ligands())
    b0 = int(bad.n_bonds_per_ligand[:6].sum())
    bad.bonds[b0] = [0, 500]          # ligand 6 (batch 1 at size 4): bond to a missing atom
    with pytest.raises(pkg.AddockError) as e:
        ctx.ad_dock_stream(bad, 4, p, 17)
    assert "batch 1" in str(e.value) and "ligand 2" in str(e.value)
    with pytest.raises(pkg.AddockError):
        ctx.ad_dock_stream(pack, 0, p, 17)


def test_dock_parameter_errors(pkg, setup):
    ctx, grid, G = setup
    batch = ctx.ad_load_ligands([synth.ligand(60, 10, 2)])
    for kw, code in [(dict(pop=1), pkg.AD_E_INVALID), (dict(pop=5000), pkg.AD_E_INVALID),
                     (dict(ls_rate=1.5), pkg.AD_E_INVALID), (dict(rho=1.0), pkg.AD_E_INVALID),
                     (dict(autostop=2), pkg.AD_E_INVALID), (dict(ls_method=2), pkg.AD_E_UNSUPPORTED),
                     (dict(ls_method=1, sw_rho=0.0), pkg.AD_E_INVALID),
                     (dict(ls_method=1, sw_max_fail=0), pkg.AD_E_INVALID),
                     (dict(autostop=1, stop_std=-1.0), pkg.AD_E_INVALID),
                     (dict(nrun=0), pkg.AD_E_INVALID)]:
        with pytest.raises(pkg.AddockError) as e:
            ctx.ad_dock_batch(batch, small_params(pkg, **kw), 1)
        assert e.value.code == code, kw
    # zero generations: only the initial population
    r = ctx.ad_dock_batch(batch, small_params(pkg, max_gens=0), 1)
    assert r["generations"][0] == 0 and r["evals"][0] == 4 * 30
    batch.free()


def test_docking_statistics_match_oracle(pkg, ff, orc):
    """Single-ligand workload (24 atoms, 5 torsions; 4 runs x pop 50 x 50
    generations, ADADELTA 300 iterations on 6%), 48 independent random
    streams (ligand ids): GPU and oracle best-energy distributions agree."""
    from scipy.stats import mannwhitneyu
    c = synth.config("single24")
    grid, rec = c["grid"], c["receptor"]
    lig = c["ligands"][0]
    G = orc.grid(grid, rec)
    ctx = pkg.create(ff, 0)
    ctx.ad_load_grids(grid, G.values())
    n_seeds = 48
    batch = ctx.ad_load_ligands([lig] * n_seeds)
    kw = dict(nrun=4, pop=50, max_gens=50, ls_rate=0.06, ls_iters=300)
    r = ctx.ad_dock_batch(batch, pkg.make_params(**kw), 7)
    L = orc.ligand(lig)
    po = oracle.make_params(**kw)
    eo = np.array([orc.dock(L, G, po, 7, k)[1].min() for k in range(n_seeds)])
    eg = r["best_energy"].astype(np.float64)
    p = mannwhitneyu(eg, eo).pvalue
    assert p > 0.01, (p, np.sort(eg), np.sort(eo))
    assert abs(np.median(eg) - np.median(eo)) < 0.3 + 0.05 * abs(np.median(eo)), (np.median(eg), np.median(eo))
    batch.free()
    ctx.close()


@pytest.mark.parametrize("cfg,max_evals", [("screen64", 20_000), ("batch4096", 3_000)])
def test_full_size_docking_rescores_at_sampled_ligands(pkg, ff, orc, cfg, max_evals):
    """A configuration's whole ligand set, receptor and grid, docked in the
    launch configuration the benchmark times (runs, population, local search,
    atom-capacity buckets, two-per-wavefront packing; only the evaluation cap
    is lower).  Every returned run energy re-scores bitwise through the score
    kernel, and the best poses of ligands sampled across the size range (packed,
    64-atom and 128-atom buckets) re-score with the oracle's energy."""
    c = synth.config(cfg)
    ligs = c["ligands"]
    ctx = pkg.create(ff, 0)
    try:
        ctx.ad_build_grids(c["grid"], c["receptor"])
        batch = ctx.ad_load_ligands(ligs)
        d = dict(c["dock"])
        d["max_evals"] = max_evals
        p = pkg.make_params(**d)
        print(f"docking {cfg}: {len(ligs)} ligands, cap {max_evals} evaluations per run", flush=True)
        r = ctx.ad_dock_batch(batch, p, c["seed"], per_run=True)
        assert ctx.ad_get_schedule()["packed_runs"] > 0
        n, nrun = r["run_energy"].shape
        assert n == len(ligs) and np.all(np.isfinite(r["run_energy"]))
        idx = np.repeat(np.arange(n, dtype=np.int32), nrun)
        Er, _, _ = ctx.ad_score_poses(batch, idx, r["run_genotype"].reshape(n * nrun, -1))
        assert np.array_equal(Er, r["run_energy"].reshape(-1))
        assert np.array_equal(r["best_energy"], r["run_energy"].min(axis=1))
        # sampled ligands: smallest, largest, and every eighth of the size order
        nat = np.asarray(ligs.n_atoms_per_ligand) if hasattr(ligs, "n_atoms_per_ligand") else np.array([l.n_atoms for l in ligs])
        order = np.argsort(nat, kind="stable")
        pick = sorted(set(order[np.linspace(0, n - 1, 9).round().astype(int)].tolist()))
        if cfg == "batch4096":
            assert nat[pick].max() > 64   # the 128-atom bucket is sampled
        assert nat[pick].min() <= 32      # so is a packed ligand
        G = orc.grid(c["grid"], c["receptor"], lazy=True)
        for i in pick:
            Eo, _, To = orc.score(orc.ligand(ligs[i]), G, r["best_genotype"][i].astype(np.float64))
            assert abs(r["best_energy"][i] - Eo) <= max(E_ABS, E_REL * abs(Eo)), (i, nat[i])
            assert abs(r["best_score"][i] - To[2]) <= max(E_ABS, E_REL * abs(To[2])), (i, nat[i])
        batch.free()
    finally:
        ctx.close()


def test_docking_extreme_ligands_and_degenerate_settings(pkg, setup, orc):
    """Ligands at the ends of every size limit (one atom, two atoms, the
    packing limits of 32 atoms / 25 torsions and one atom past them, 64 and 65
    atoms, the 128-atom maximum with 32 torsions) docked with degenerate
    search settings: a single run with a population of two and one local
    search per generation (an idle packed half), local searches of zero
    iterations, and a cap below one population (initial population only)."""
    ctx, grid, G = setup
    # random trees of 32 atoms have about 20 eligible torsions: zigzag chains
    # reach the torsion limit of packing (25) and pass it (26)
    spec = [(1, 0), (2, 0), (32, 25), (32, 26), (33, 20), (64, 32), (65, 32), (128, 32)]
    ligs = [chain_ligand(n, t) if n == 32 else synth.ligand(140 + i, n, t) for i, (n, t) in enumerate(spec)]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    assert [L.n_tor for L in OL[2:4]] == [25, 26]
    packable = sum(l.n_atoms <= 32 and L.n_tor <= 25 for l, L in zip(ligs, OL))
    cases = [(dict(nrun=1, pop=2, ls_rate=0.5, max_gens=3, ls_iters=20), 2 + 3 * (1 + 1 * 20)),
             (dict(nrun=3, pop=5, ls_rate=0.4, max_gens=2, ls_iters=0), 5 + 2 * (4 + 2 * 0)),
             (dict(nrun=2, pop=10, max_gens=5, max_evals=9), 10)]
    for kw, per_run_evals in cases:
        print("case", kw, flush=True)
        r = ctx.ad_dock_batch(batch, small_params(pkg, **kw), 5, per_run=True)
        nrun = kw["nrun"]
        assert ctx.ad_get_schedule()["packed_runs"] == (nrun * packable if kw.get("ls_iters", 40) > 0 else 0), kw
        assert np.all(r["evals"] == nrun * per_run_evals), kw
        assert np.all(np.isfinite(r["run_energy"])), kw
        for l in range(len(ligs)):
            Er, _, _ = ctx.ad_score_poses(batch, np.full(nrun, l, np.int32), r["run_genotype"][l])
            assert np.array_equal(Er, r["run_energy"][l]), (kw, spec[l])
            Eo, _, To = orc.score(OL[l], G, r["best_genotype"][l].astype(np.float64))
            if abs(r["best_energy"][l] - Eo) > max(E_ABS, E_REL * abs(Eo)):
                # what a reader needs to judge a miss: the pose, and the oracle's
                # energy of it again and from a freshly prepared ligand
                Ea = orc.score(OL[l], G, r["best_genotype"][l].astype(np.float64))[0]
                Ef = orc.score(orc.ligand(ligs[l]), G, r["best_genotype"][l].astype(np.float64))[0]
                pytest.fail(f"{kw} {spec[l]}: gpu {r['best_energy'][l]!r} oracle {Eo!r} (again {Ea!r}, fresh "
                            f"ligand {Ef!r}) genotype {r['best_genotype'][l].tobytes().hex()}")
            assert abs(r["best_score"][l] - To[2]) <= max(E_ABS, E_REL * abs(To[2])), (kw, spec[l])
    batch.free()
