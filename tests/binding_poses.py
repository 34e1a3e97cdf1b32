"""Binding-regime poses for parity tests, generated with the FP64 oracle alone.

Random poses of a ligand in a receptor are almost all clashes (|E| of 1e4 to
1e8 kcal/mol), where the energy bound max(1e-3, 1e-5 |E|) admits errors of
whole kcal/mol.  Docked poses sit at |E| <= 100 kcal/mol, where the same bound
is 1e-3 kcal/mol.  These poses come from the oracle's ADADELTA (FP64) started
near a binding site: a seeded pocket for small ligands, the face of a slab of
receptor atoms for large ones (a ligand of 100 atoms does not fit a pocket of
5-7 A radius).  Ligands are drawn with a 2.5 A minimum distance between atoms
three or more bonds apart, so that large ones are not strained in their
reference conformation.  The searches run for 20, 60 or 150 iterations, so the
set mixes poses near a minimum (small gradient) with poses on the way to one.
Nothing here touches the GPU path.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import synth

E_MAX = 100.0


def slab_receptor(seed, n_atoms, side):
    """Receptor atoms of a cube of side `side` (no pocket) with z < 0: a flat
    face at z = 0 that ligands of any size can lie on."""
    r = synth.receptor(seed, 2 * n_atoms, side=side, n_pocket_spheres=0)
    keep = r.xyz[:, 2] < 0
    xyz, ty, q = r.xyz[keep][:n_atoms], r.types[keep][:n_atoms], r.charges[keep][:n_atoms]
    return synth.Receptor(xyz.astype(np.float32), ty.astype(np.int32), (q - q.mean()).astype(np.float32), [])


def site(orc, kind):
    """(grid, oracle maps, site centre, start spread) of a binding site:
    'pocket' (1,500 atoms in an 18 A cube around a pocket, 40^3 grid) or
    'slab' (1,500 atoms below z = 0, 48^3 grid centred 3 A above the face)."""
    if kind == "pocket":
        rec = synth.receptor(11, 1500, side=18.0)
        grid = synth.make_grid(40, 0.375, map_types=synth.SIX_TYPES)
        return grid, orc.grid(grid, rec), np.asarray(grid.center), 1.0
    rec = slab_receptor(5, 1500, 22.0)
    grid = synth.make_grid(48, 0.375, center=(0.0, 0.0, 3.0), map_types=synth.SIX_TYPES)
    return grid, orc.grid(grid, rec), np.array([0.0, 0.0, 4.5]), 1.5


def ligands(sizes, seed0):
    return [synth.ligand(seed0 + i, n, t, min_nonlocal=2.5) for i, (n, t) in enumerate(sizes)]


def generate(orc, OL, G, center, spread, n_target, seed, pairs=False, threads=8):
    """At least n_target poses (float32 genotypes) with |E_oracle| <= E_MAX.

    Returns (lig_idx int32 [n], genotypes float32 [n, 40], E_oracle [n]) with
    the energy of the float32 genotype.  pairs=True: poses 2w and 2w + 1 name
    the same ligand and are kept or dropped together (the packed shape).
    """
    rng = np.random.default_rng(seed)
    P = oracle.make_params()
    idx, genos, energies = [], [], []
    for _round in range(20):
        if sum(len(a) for a in idx) >= n_target:
            break
        jobs = []
        for k in range(max(64, n_target) // 2 * 2):
            i = int((k // 2 if pairs else k) % len(OL))
            g = np.zeros(synth.GENO_STRIDE)
            g[:3] = center + rng.normal(0.0, spread, 3)
            q = rng.normal(size=4)
            g[3:7] = q / np.linalg.norm(q)
            g[7:7 + OL[i].n_tor] = rng.normal(0.0, 0.3, OL[i].n_tor)
            jobs.append((i, g, int(rng.choice([20, 60, 150]))))
        with ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(lambda j: orc.adadelta(OL[j[0]], G, P, j[1], j[2])[0], jobs))
        li = np.array([j[0] for j in jobs], np.int32)
        gf = np.array(res, np.float32)
        E, _, _ = orc.score_batch(OL, li, G, gf, grad=False)
        ok = np.abs(E) <= E_MAX
        if pairs:   # keep poses 2w and 2w + 1 (one ligand) only together
            ok = np.repeat(ok.reshape(-1, 2).all(axis=1), 2)
        idx.append(li[ok])
        genos.append(gf[ok])
        energies.append(E[ok])
    assert sum(len(a) for a in idx) >= n_target, "could not find enough binding-regime poses"
    return np.concatenate(idx), np.concatenate(genos), np.concatenate(energies)
