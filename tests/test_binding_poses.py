"""The binding-regime pose sets of the GPU parity tests exist and are what
they claim (CPU, oracle only): enough poses per size class, every one with
|E| <= 100 kcal/mol and finite gradient, deterministic for a seed, packed
pairs of one ligand, and a spread of gradient sizes (poses near a minimum
and poses on the way to one)."""
import numpy as np
import pytest

import binding_poses as bp


@pytest.mark.parametrize("kind,sizes,pairs", [
    ("pocket", [(12, 2), (20, 4), (26, 9), (32, 25), (32, 8), (16, 0)], True),
    ("slab", [(40, 8), (48, 10), (56, 12), (64, 16), (33, 3), (60, 30)], False),
    ("slab", [(70, 16), (90, 24), (110, 28), (128, 32), (65, 0), (100, 10)], False),
])
def test_binding_pose_sets(orc, kind, sizes, pairs):
    grid, G, c, s = bp.site(orc, kind)
    OL = [orc.ligand(l) for l in bp.ligands(sizes, 100)]
    idx, g, E = bp.generate(orc, OL, G, c, s, 500, 7, pairs=pairs)
    assert len(idx) >= 500
    Eo, Go, _ = orc.score_batch(OL, idx, G, g)
    assert np.array_equal(Eo, E) and np.all(np.abs(Eo) <= bp.E_MAX)
    assert np.all(np.isfinite(Go))
    gn = np.linalg.norm(Go, axis=1)
    assert gn.min() < 20.0 and np.percentile(gn, 90) > 2 * gn.min()
    for i, L in enumerate(OL):
        assert (idx == i).sum() >= 20, i
    if pairs:
        assert len(idx) % 2 == 0 and np.all(idx[0::2] == idx[1::2])
    idx2, g2, _ = bp.generate(orc, OL, G, c, s, 500, 7, pairs=pairs)
    assert np.array_equal(idx, idx2) and np.array_equal(g, g2)
