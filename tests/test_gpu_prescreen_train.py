"""The pre-screen trained on the GPU by its own kernels, on docking labels
the plain method produces, and what it gains over screening without it.

Labels: best energies of 8,192 synthetic ligands (atoms lognormal 10-100,
torsions 0-32) docked by ad_dock_batch (5 runs x population 100, 10
generations) against the 8,000-atom receptor on its 64^3 grid; 6,144 train,
2,048 held out.  Gain: of the held-out plain top 5% (102 ligands), the share
found in the pre-screen's top 20% must beat random selection (20%) by far and
beat ranking by ligand size; the rank correlation must be clearly positive.
Training is stochastic, so only these gain statistics are checked; the
trained weights are not pinned.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03678_amd as pkg
    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def setup(pkg, ff):
    ctx = pkg.create(ff, 0)
    ctx.ad_build_grids(synth.make_grid(64, 0.375, map_types=synth.ALL_TYPES), synth.receptor(20200707, 8000))
    ligs = synth.ligand_set_fast(4242, 8192, atoms=(10, 100), torsions=(0, 32), dist="lognormal")
    batch = ctx.ad_load_ligands(ligs)
    p = pkg.make_params(nrun=5, pop=100, max_gens=10, ls_rate=0.06, ls_iters=300)
    y = ctx.ad_dock_batch(batch, p, seed=3)["best_energy"].astype(np.float64)
    yield ctx, ligs, batch, y
    batch.free()
    ctx.close()


def test_training_reduces_the_loss_and_ranks_held_out_ligands(pkg, setup):
    from scipy.stats import spearmanr
    from paper_2007_03678_amd import screen
    ctx, ligs, batch, y = setup
    assert np.all(np.isfinite(y))
    perm = np.random.default_rng(0).permutation(len(ligs))
    ho, tr = perm[:2048].astype(np.int32), perm[2048:].astype(np.int32)
    ps = pkg.Prescreen(ctx, seed=1, label_max=0.0)
    curve = ps.ad_prescreen_train(batch, tr, y[tr], epochs=20, seed=2)
    print("loss curve", np.round(curve, 3))
    assert np.all(np.isfinite(curve))
    assert curve[-1] < 0.7 * curve[0]
    pred = ps.ad_prescreen_predict(batch, ho)
    rho = spearmanr(pred, y[ho])[0]
    sel = screen.top_fraction(pred, 0.2)
    hits, pos = screen.recall(y[ho], sel, top_frac=0.05)
    nat = np.array([ligs[i].n_atoms for i in ho], dtype=np.float64)
    size_hits, _ = screen.recall(y[ho], screen.top_fraction(-nat, 0.2), top_frac=0.05)
    print(f"spearman {rho:.3f}; recall of top 5% in top 20%: pre-screen {hits}/{pos}, size {size_hits}/{pos}")
    assert rho > 0.5
    assert hits >= 2.5 * 0.2 * pos          # at least 2.5x random selection
    assert hits > size_hits
    # predictions are deterministic for fixed weights
    assert np.array_equal(pred, ps.ad_prescreen_predict(batch, ho))
    ps.close()


def test_tail_focused_labels_find_the_best_ligands(pkg, setup):
    """Labels clipped at their 10th percentile (the campaign's setting: the
    network orders the best labels and the rest count as equal) find more of
    the held-out top 2 % within the predicted top 10 % than labels clipped at
    0 kcal/mol.  At this size (6,144 training ligands) the gain is small; at
    the campaign's 200,000 it is large (measured by the bench)."""
    from paper_2007_03678_amd import screen
    ctx, ligs, batch, y = setup
    perm = np.random.default_rng(0).permutation(len(ligs))
    ho, tr = perm[:2048].astype(np.int32), perm[2048:].astype(np.int32)
    found = {}
    for name, lm in (("q10", float(np.percentile(y[tr], 10))), ("zero", 0.0)):
        ps = pkg.Prescreen(ctx, seed=1, label_max=lm)
        ps.ad_prescreen_train(batch, tr, y[tr], epochs=20, seed=2)
        pred = ps.ad_prescreen_predict(batch, ho)
        found[name] = screen.recall(y[ho], screen.top_fraction(pred, 0.1), top_frac=0.02)
        ps.close()
    print("top 2 % in top 10 %:", found)
    (h_q, pos), (h_z, _) = found["q10"], found["zero"]
    assert h_q >= 0.5 * pos          # five times random selection
    assert h_q >= h_z                # training is bitwise reproducible, so this is a fixed comparison


def test_training_is_reproducible(pkg, setup):
    ctx, ligs, batch, y = setup
    idx = np.arange(512, dtype=np.int32)
    w = []
    for _ in range(2):
        ps = pkg.Prescreen(ctx, seed=5, batch_size=64, label_max=0.0)
        ps.ad_prescreen_train(batch, idx, y[idx], epochs=2, seed=9)
        w.append(ps.ad_prescreen_get_params())
        ps.close()
    assert np.array_equal(w[0], w[1])
