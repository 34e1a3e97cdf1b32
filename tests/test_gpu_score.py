"""GPU parity of the hot path (score + gradient) against the FP64 oracle.

Every call goes through the C ABI.  Tolerances (per pose):
  energy:   |E_gpu - E_oracle| <= max(1e-3, 1e-5 |E_oracle|)   kcal/mol
  gradient: ||g_gpu - g_oracle||_2 <= 1e-4 max(||g_oracle||_2, 1), and the
            same bound on the torsion sub-vector alone.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

E_ABS, E_REL, G_REL = 1e-3, 1e-5, 1e-4


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


def check_parity(E, Gr, T, Eo, Go, To, n_tor, label=""):
    E = np.asarray(E, np.float64)
    tol = np.maximum(E_ABS, E_REL * np.abs(Eo))
    bad = np.abs(E - Eo) > tol
    assert not bad.any(), (label, np.where(bad)[0][:5], E[bad][:5], Eo[bad][:5])
    if T is not None:
        for c in range(3):
            tc = np.maximum(E_ABS, E_REL * np.abs(To[:, c]))
            assert np.all(np.abs(T[:, c] - To[:, c]) <= tc), (label, c)
    if Gr is not None:
        for p in range(len(E)):
            d = Gr[p].astype(np.float64) - Go[p]
            scale = max(np.linalg.norm(Go[p]), 1.0)
            assert np.linalg.norm(d) <= G_REL * scale, (label, p, np.linalg.norm(d) / scale)
            k = n_tor[p]
            if k:
                st = max(np.linalg.norm(Go[p, 7:7 + k]), 1.0)
                assert np.linalg.norm(d[7:7 + k]) <= G_REL * st, (label, p, "torsions")
            assert np.all(Gr[p, 7 + k:] == 0) and Gr[p, 6] == 0


SIZES = [(1, 0), (2, 0), (4, 1), (15, 3), (24, 5), (37, 9), (60, 15), (64, 16), (65, 20), (100, 32), (128, 32)]


@pytest.fixture(scope="module")
def shared_maps(orc):
    """One receptor and its oracle maps, loaded identically into both sides."""
    rec = synth.receptor(11, 1500, side=18.0)
    grid = synth.make_grid(40, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    return grid, G


def test_score_parity_identical_maps(ctx, orc, shared_maps):
    grid, G = shared_maps
    ctx.ad_load_grids(grid, G.values())
    ligs = [synth.ligand(300 + i, n, t, shuffle=(i % 2 == 1)) for i, (n, t) in enumerate(SIZES)]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    for i, l in enumerate(ligs):
        info = batch.info(i)
        assert info["n_atoms"] == l.n_atoms and info["n_torsions"] == OL[i].n_tor
        assert info["n_pairs"] == OL[i].n_pairs and info["n_fragments"] == OL[i].n_frag
    rng = np.random.default_rng(1)
    n = 1500
    idx = rng.integers(0, len(ligs), size=n).astype(np.int32)
    ntor = np.array([OL[i].n_tor for i in idx])
    genos = synth.random_genotypes(2, n, ntor, grid, margin=1.0, outside_frac=0.1)
    E, Gr, T = ctx.ad_score_poses(batch, idx, genos, grad=True, terms=True)
    Eo, Go, To = orc.score_batch(OL, idx, G, genos)
    check_parity(E, Gr, T, Eo, Go, To, ntor, "random poses")
    # energy-only kernel gives the same energies
    E2, _, _ = ctx.ad_score_poses(batch, idx, genos, grad=False)
    assert np.array_equal(E, E2)
    batch.free()


def test_score_parity_near_pocket(ctx, orc, shared_maps):
    """Low-energy region: poses around the pocket centre, unit quaternions."""
    grid, G = shared_maps
    ctx.ad_load_grids(grid, G.values())
    ligs = [synth.ligand(400 + i, n, t) for i, (n, t) in enumerate([(20, 4), (32, 8), (48, 12)])]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    small = synth.make_grid(8, 0.5, center=grid.center)
    n = 600
    idx = np.arange(n, dtype=np.int32) % 3
    ntor = np.array([OL[i].n_tor for i in idx])
    genos = synth.random_genotypes(3, n, ntor, small, normalize_q=True)
    # small torsion angles keep the reference conformation (few intramolecular clashes)
    genos[:, 7:] *= 0.2
    E, Gr, T = ctx.ad_score_poses(batch, idx, genos, grad=True, terms=True)
    Eo, Go, To = orc.score_batch(OL, idx, G, genos)
    check_parity(E, Gr, T, Eo, Go, To, ntor, "pocket poses")
    batch.free()


def test_identity_genotype_gives_reference_energy_and_nan_handling(ctx, orc, shared_maps):
    grid, G = shared_maps
    ctx.ad_load_grids(grid, G.values())
    lig = synth.ligand(501, 30, 6)
    batch = ctx.ad_load_ligands([lig])
    L = orc.ligand(lig)
    g = np.zeros((4, 40), np.float32)
    g[:, 0:3] = np.array(grid.center, np.float32)
    g[:, 3] = 1.0
    g[1, 7] = np.nan
    g[2, 0] = np.inf
    g[3, 3:7] = [0.0, 0.0, 0.0, 2.0]
    E, Gr, T = ctx.ad_score_poses(batch, np.zeros(4, np.int32), g, grad=True, terms=True)
    Eo, Go, To = orc.score(L, G, g[0].astype(np.float64))
    assert abs(E[0] - Eo) <= max(E_ABS, E_REL * abs(Eo))
    assert np.isnan(E[1]) and np.isnan(Gr[1]).all() and np.isnan(T[1]).all()
    assert np.isnan(E[2])
    assert np.isfinite(E[3])
    batch.free()


def test_device_pointer_path_and_determinism(pkg, ctx, orc, shared_maps):
    import torch
    grid, G = shared_maps
    ctx.ad_load_grids(grid, torch.from_numpy(G.values()).cuda())
    ligs = [synth.ligand(600 + i, n, t) for i, (n, t) in enumerate([(24, 5), (90, 25)])]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    n = 4096
    idx = (np.arange(n) % 2).astype(np.int32)
    ntor = np.array([OL[i].n_tor for i in idx])
    genos = synth.random_genotypes(4, n, ntor, grid, margin=1.5)
    gd = torch.from_numpy(genos).cuda()
    idd = torch.from_numpy(idx).cuda()
    E1, G1, T1 = ctx.ad_score_poses(batch, idd, gd, grad=True, terms=True)
    ctx.ad_synchronize()
    E2, G2, T2 = ctx.ad_score_poses(batch, idd, gd, grad=True, terms=True)
    ctx.ad_synchronize()
    assert torch.equal(E1, E2) and torch.equal(G1, G2) and torch.equal(T1, T2)
    Eh, Gh, Th = ctx.ad_score_poses(batch, idx, genos, grad=True, terms=True)
    assert np.array_equal(E1.cpu().numpy(), Eh) and np.array_equal(G1.cpu().numpy(), Gh)
    sel = np.arange(0, n, 16)
    Eo, Go, To = orc.score_batch(OL, idx[sel], G, genos[sel])
    check_parity(Eh[sel], Gh[sel], Th[sel], Eo, Go, To, ntor[sel], "device path")
    # device-side bad ligand index -> NaN, not a fault
    bad = torch.tensor([5, -1, 0], dtype=torch.int32, device="cuda")
    Eb, _, _ = ctx.ad_score_poses(batch, bad, gd[:3])
    ctx.ad_synchronize()
    Eb = Eb.cpu().numpy()
    assert np.isnan(Eb[0]) and np.isnan(Eb[1]) and np.isfinite(Eb[2])
    batch.free()


def test_host_argument_errors(pkg, ctx, shared_maps):
    grid, G = shared_maps
    ctx.ad_load_grids(grid, G.values())
    batch = ctx.ad_load_ligands([synth.ligand(700, 12, 2)])
    g = np.zeros((1, 40), np.float32)
    g[0, 3] = 1
    with pytest.raises(pkg.AddockError) as e:
        ctx.ad_score_poses(batch, np.array([1], np.int32), g)
    assert e.value.code == pkg.AD_E_INVALID
    # ligand with a type that has no map -> AD_E_NOMAP
    lig = synth.ligand(701, 12, 2)
    lig.types[0] = synth.TYPE_ID["SA"]
    with pytest.raises(pkg.AddockError) as e:
        ctx.ad_load_ligands([lig])
    assert e.value.code == pkg.AD_E_NOMAP
    batch.free()


def test_gpu_maps_match_oracle_maps(ctx, orc):
    rec = synth.receptor(21, 900, side=16.0)
    grid = synth.make_grid((30, 26, 22), 0.4, map_types=synth.ALL_TYPES)
    M = ctx.ad_build_grids(grid, rec, want_maps=True)
    Mo = orc.grid(grid, rec).values()
    rel = np.abs(M - Mo) / np.maximum(1.0, np.abs(Mo))
    assert rel.max() <= 1e-6, rel.max()
    assert (M == Mo).mean() > 0.99


def test_state_errors(pkg, ff):
    c = pkg.create(ff, 0)
    with pytest.raises(pkg.AddockError) as e:
        c.ad_load_ligands([synth.ligand(1, 10, 2)])
    assert e.value.code == pkg.AD_E_STATE
    c.close()


@pytest.mark.parametrize("cfg", ["single24", "screen64", "batch4096", "campaign"])
def test_full_size_sampled_parity(ctx, orc, cfg):
    """Paper-scale receptor and grid (40^3 to 126^3 nodes): GPU-built maps,
    oracle maps computed lazily at the nodes the sampled poses touch; the
    ligands are the first 8 of each configuration's set."""
    c = synth.config(cfg, n_ligands=8)
    grid, rec = c["grid"], c["receptor"]
    ctx.ad_build_grids(grid, rec)
    ligs = c["ligands"]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    G = orc.grid(grid, rec, lazy=True)
    n = 2048
    idx = (np.arange(n) % len(ligs)).astype(np.int32)
    ntor = np.array([OL[i].n_tor for i in idx])
    genos = synth.random_genotypes(9, n, ntor, grid, margin=2.0)
    E, Gr, T = ctx.ad_score_poses(batch, idx, genos, grad=True, terms=True)
    sel = np.arange(0, n, 32)
    Eo, Go, To = orc.score_batch(OL, idx[sel], G, genos[sel])
    check_parity(E[sel], Gr[sel], T[sel], Eo, Go, To, ntor[sel], cfg)
    batch.free()
