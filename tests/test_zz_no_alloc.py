"""ad_score_poses_noalloc: the allocation-free variant of ad_score_poses.

It stages host buffers through the library's static device block instead of
the context's staging buffer and runs the same kernels, so its outputs must
equal ad_score_poses' (host buffers) bit for bit.  Two calls in a row, the
second smaller, check that nothing of an earlier call leaks into a later one;
a few poses are also held to the oracle's tolerance (energy max(1e-3, 1e-5|E|)
kcal/mol, gradient 1e-4 relative).
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
def setup(pkg, ff, orc):
    rec = synth.receptor(21, 1200, side=16.0)
    grid = synth.make_grid(32, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    ctx = pkg.create(ff, 0)
    ctx.ad_load_grids(grid, G.values())
    small = [synth.ligand(31 + k, n, t) for k, (n, t) in enumerate([(9, 2), (24, 5), (40, 9), (64, 16)])]
    large = small + [synth.ligand(41, 100, 30)]
    bs, bl = ctx.ad_load_ligands(small), ctx.ad_load_ligands(large)
    yield pkg, ctx, grid, G, small, large, bs, bl
    bs.free()
    bl.free()
    ctx.close()


def _same(a, b):
    return a.shape == b.shape and np.array_equal(a, b, equal_nan=True)


def _poses(seed, n, ligs, grid):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(ligs), n).astype(np.int32)
    genos = synth.random_genotypes(seed + 1, n, [ligs[i].n_torsions for i in idx], grid, margin=2.0)
    return idx, genos


@pytest.mark.parametrize("which", ["wave64", "wave128"])
def test_noalloc_equals_score_poses_on_two_calls(setup, which):
    pkg, ctx, grid, G, small, large, bs, bl = setup
    ligs, batch = (small, bs) if which == "wave64" else (large, bl)
    print("noalloc vs ad_score_poses:", which, flush=True)
    for call, n in enumerate([pkg.NOALLOC_MAX_POSES, 257]):
        idx, genos = _poses(100 * call + len(ligs), n, ligs, grid)
        E0, G0, T0 = ctx.ad_score_poses(batch, idx, genos, grad=True, terms=True)
        E1, G1, T1 = ctx.ad_score_poses_noalloc(batch, idx, genos, grad=True, terms=True)
        assert _same(E0, E1) and _same(G0, G1) and _same(T0, T1), (which, call, n)
        # energy only (no gradient / terms sections requested)
        E2, _, _ = ctx.ad_score_poses(batch, idx, genos)
        E3, G3, T3 = ctx.ad_score_poses_noalloc(batch, idx, genos)
        assert G3 is None and T3 is None
        assert _same(E2, E3), (which, call, n, "energy only")


def test_noalloc_matches_the_oracle(setup, orc):
    pkg, ctx, grid, G, small, large, bs, bl = setup
    idx, genos = _poses(7, 48, large, grid)
    E, Gr, _ = ctx.ad_score_poses_noalloc(bl, idx, genos, grad=True)
    OL = [orc.ligand(l) for l in large]
    Eo, Go, _ = orc.score_batch(OL, idx, G, genos)
    assert np.all(np.abs(E - Eo) <= np.maximum(1e-3, 1e-5 * np.abs(Eo)))
    for p in range(len(E)):
        assert np.linalg.norm(Gr[p] - Go[p]) <= 1e-4 * max(np.linalg.norm(Go[p]), 1.0), p


def test_noalloc_rejects_more_than_its_static_limit(setup):
    pkg, ctx, grid, G, small, large, bs, bl = setup
    idx, genos = _poses(3, pkg.NOALLOC_MAX_POSES + 1, small, grid)
    with pytest.raises(pkg.AddockError) as e:
        ctx.ad_score_poses_noalloc(bs, idx, genos)
    assert e.value.code == pkg.AD_E_INVALID and "static limit" in str(e.value)
    # an empty call is a no-op; a bad index is rejected on the host
    E, _, _ = ctx.ad_score_poses_noalloc(bs, idx[:0], genos[:0])
    assert E.shape == (0,)
    bad = idx[:4].copy()
    bad[2] = len(small)
    with pytest.raises(pkg.AddockError):
        ctx.ad_score_poses_noalloc(bs, bad, genos[:4])
