"""GPU parity in the binding regime, for every evaluation shape.

Each set holds at least 500 poses with |E_oracle| <= 100 kcal/mol from the
oracle's own ADADELTA (tests/binding_poses.py), so the energy bound
max(1e-3, 1e-5 |E|) is 1e-3 kcal/mol for every pose.  Every pose is compared
element by element: energy, the three score terms, and the gradient
(||g_gpu - g_oracle|| <= 1e-4 max(||g_oracle||, 1), also on the torsion
sub-vector alone) through the C ABI with the shape forced:

  - AD_SHAPE_WAVE64: one wavefront per pose (ligands of 33-64 atoms on the
    slab face; ligands of up to 32 atoms in the pocket);
  - AD_SHAPE_WAVE128: two atoms per lane (ligands of 65-128 atoms on the slab
    face, and the 33-64-atom set through the same kernel);
  - AD_SHAPE_PACKED: two poses per wavefront, the evaluation the docking
    search's packed local search runs (ligands of up to 32 atoms and 25
    torsions), pairs of different poses of one ligand;
and the packed local search after 1 and 3 ADADELTA iterations against the
oracle's from the same starts.
"""
import numpy as np
import pytest

import binding_poses as bp
import oracle
import synth

pytestmark = pytest.mark.gpu

E_ABS, E_REL, G_REL = 1e-3, 1e-5, 1e-4

SMALL = [(12, 2), (20, 4), (26, 9), (32, 25), (32, 8), (16, 0)]
MID = [(40, 8), (48, 10), (56, 12), (64, 16), (33, 3), (60, 30)]
LARGE = [(70, 16), (90, 24), (110, 28), (128, 32), (65, 0), (100, 10)]


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03678_amd as pkg
    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def ctx(pkg, ff):
    c = pkg.create(ff, 0)
    yield c
    c.close()


def poses(orc, kind, sizes, seed0, seed, pairs=False):
    grid, G, c, s = bp.site(orc, kind)
    ligs = bp.ligands(sizes, seed0)
    OL = [orc.ligand(l) for l in ligs]
    idx, g, _ = bp.generate(orc, OL, G, c, s, 500, seed, pairs=pairs)
    return grid, G, ligs, OL, idx, g


def check(E, Gr, T, Eo, Go, To, ntor, label):
    E = np.asarray(E, np.float64)
    assert np.all(np.abs(Eo) <= bp.E_MAX)
    dE = np.abs(E - Eo)
    tol = np.maximum(E_ABS, E_REL * np.abs(Eo))
    assert np.all(dE <= tol), (label, np.where(dE > tol)[0][:5], float(np.max(dE)))
    for c in range(3):
        assert np.all(np.abs(T[:, c] - To[:, c]) <= np.maximum(E_ABS, E_REL * np.abs(To[:, c]))), (label, c)
    worst = 0.0
    for p in range(len(E)):
        d = Gr[p].astype(np.float64) - Go[p]
        r = np.linalg.norm(d) / max(np.linalg.norm(Go[p]), 1.0)
        k = ntor[p]
        rt = np.linalg.norm(d[7:7 + k]) / max(np.linalg.norm(Go[p, 7:7 + k]), 1.0) if k else 0.0
        worst = max(worst, r, rt)
        assert r <= G_REL and rt <= G_REL, (label, p, r, rt)
        assert Gr[p, 6] == 0 and np.all(Gr[p, 7 + k:] == 0)
    print(f"{label}: {len(E)} poses, max |dE| {np.max(dE):.2e}, max gradient rel {worst:.2e}", flush=True)


def score_and_check(pkg, ctx, orc, grid, G, ligs, OL, idx, g, shape, label):
    ctx.ad_load_grids(grid, G.values())
    batch = ctx.ad_load_ligands(ligs)
    try:
        E, Gr, T = ctx.ad_score_poses(batch, idx, g, grad=True, terms=True, shape=shape)
        Eo, Go, To = orc.score_batch(OL, idx, G, g)
        check(E, Gr, T, Eo, Go, To, np.array([OL[i].n_tor for i in idx]), label)
        E2, _, _ = ctx.ad_score_poses(batch, idx, g, shape=shape)   # energy-only variant: same energies
        assert np.array_equal(E, E2), label
    finally:
        batch.free()


def test_binding_parity_wave64(pkg, ctx, orc):
    for kind, sizes, s0 in (("slab", MID, 100), ("pocket", SMALL, 120)):
        grid, G, ligs, OL, idx, g = poses(orc, kind, sizes, s0, 11)
        score_and_check(pkg, ctx, orc, grid, G, ligs, OL, idx, g, pkg.SHAPE_WAVE64, f"wave64/{kind}")


def test_binding_parity_wave128(pkg, ctx, orc):
    for sizes, s0 in ((LARGE, 140), (MID, 100)):
        grid, G, ligs, OL, idx, g = poses(orc, "slab", sizes, s0, 12)
        score_and_check(pkg, ctx, orc, grid, G, ligs, OL, idx, g, pkg.SHAPE_WAVE128, f"wave128/{sizes[0][0]}")


def test_binding_parity_packed(pkg, ctx, orc):
    grid, G, ligs, OL, idx, g = poses(orc, "pocket", SMALL, 120, 13, pairs=True)
    assert np.all(idx[0::2] == idx[1::2]) and np.any(g[0::2] != g[1::2])
    score_and_check(pkg, ctx, orc, grid, G, ligs, OL, idx, g, pkg.SHAPE_PACKED, "packed")


def test_packed_and_wave64_local_search_follow_oracle(pkg, ctx, orc):
    """ADADELTA from binding-regime starts, 1 and 3 iterations, packed and one
    per wavefront: the best pose and its energy follow the FP64 oracle's."""
    grid, G, ligs, OL, idx, g = poses(orc, "pocket", SMALL, 120, 14, pairs=True)
    idx, g = idx[:256], g[:256]
    ctx.ad_load_grids(grid, G.values())
    batch = ctx.ad_load_ligands(ligs)
    try:
        p = pkg.make_params()
        for iters in (1, 3):
            ref = [orc.adadelta(OL[i], G, oracle.make_params(), g[k].astype(np.float64), iters)
                   for k, i in enumerate(idx)]
            for shape in (pkg.SHAPE_PACKED, pkg.SHAPE_WAVE64):
                g1, E1 = ctx.ad_local_search(batch, idx, g, p, iters, shape=shape)
                for k in range(len(idx)):
                    bo, Eo = ref[k]
                    assert abs(E1[k] - Eo) <= max(1e-3, 1e-5 * abs(Eo)), (shape, iters, k, E1[k], Eo)
                    assert np.allclose(g1[k][:7 + OL[idx[k]].n_tor], bo[:7 + OL[idx[k]].n_tor], atol=1e-4), \
                        (shape, iters, k)
                # the returned pose re-scores to the returned energy through the same shape
                Er, _, _ = ctx.ad_score_poses(batch, idx, g1, shape=shape)
                assert np.array_equal(Er, E1), (shape, iters)
    finally:
        batch.free()


def test_shape_validation(pkg, ctx, orc):
    grid, G, c, s = bp.site(orc, "pocket")
    ctx.ad_load_grids(grid, G.values())
    # a zigzag chain of 30 atoms with 26 rotatable bonds: over the packed torsion limit
    x = np.zeros((30, 3), np.float32)
    x[:, 0] = 1.26 * np.arange(30)
    x[1::2, 1] = 0.8
    chain = synth.Ligand(np.zeros(30, np.int32), np.zeros(30, np.float32), x,
                         np.array([[i, i + 1] for i in range(29)], np.int32),
                         np.array([0] + [1] * 26 + [0, 0], np.uint8))
    ligs = bp.ligands([(20, 4), (40, 8)], 300) + [chain]
    assert chain.n_torsions == 26
    batch = ctx.ad_load_ligands(ligs)
    try:
        g = np.zeros((2, 40), np.float32)
        g[:, :3] = grid.center
        g[:, 3] = 1.0
        for idx, shape in (([1, 1], pkg.SHAPE_PACKED), ([2, 2], pkg.SHAPE_PACKED), ([0, 1], pkg.SHAPE_PACKED),
                           ([0, 0], 7)):
            with pytest.raises(pkg.AddockError):
                ctx.ad_score_poses(batch, np.array(idx, np.int32), g, shape=shape)
        # an odd count leaves the last half idle; the pose still scores
        E, _, _ = ctx.ad_score_poses(batch, np.zeros(1, np.int32), g[:1], shape=pkg.SHAPE_PACKED)
        E64, _, _ = ctx.ad_score_poses(batch, np.zeros(1, np.int32), g[:1], shape=pkg.SHAPE_WAVE64)
        assert abs(E[0] - E64[0]) <= max(1e-3, 1e-5 * abs(E64[0]))
    finally:
        batch.free()
