"""Seeded synthetic inputs for the docking hot path.

This module is shared by the FP64 oracle tests and by the GPU path. It holds
only *inputs*: the force-field parameter table (data), synthetic receptors,
ligands (typed trees with 3-D reference coordinates), grid descriptions and
random genotypes.  It contains none of the scoring or search arithmetic: no pair
potentials, no map sums, no pose construction, no gradients.

Every generator takes an integer seed and is deterministic (numpy PCG64).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Force-field parameter table (AD4 functional form; values are a frozen
# synthetic table in the magnitudes of the published AD4.1 set).
# Columns: name, R_ii (A), eps_ii (kcal/mol), V (A^3), solpar, hb role
# (0 none, 1 donor, 2 acceptor), R_hb (A), eps_hb (kcal/mol).
# ---------------------------------------------------------------------------
TYPE_TABLE = [
    ("C", 4.00, 0.150, 33.51, -0.00143, 0, 0.0, 0.0),
    ("A", 4.00, 0.150, 33.51, -0.00052, 0, 0.0, 0.0),
    ("N", 3.50, 0.160, 22.45, -0.00162, 0, 0.0, 0.0),
    ("NA", 3.50, 0.160, 22.45, -0.00162, 2, 1.9, 5.0),
    ("OA", 3.20, 0.200, 17.16, -0.00251, 2, 1.9, 5.0),
    ("S", 4.00, 0.200, 33.51, -0.00214, 0, 0.0, 0.0),
    ("SA", 4.00, 0.200, 33.51, -0.00214, 2, 2.5, 1.0),
    ("HD", 2.00, 0.020, 0.00, 0.00051, 1, 0.0, 0.0),
]
TYPE_NAMES = [row[0] for row in TYPE_TABLE]
TYPE_ID = {name: i for i, name in enumerate(TYPE_NAMES)}

# Global scalars of the functional form (data only).
FF_SCALARS = dict(
    w_vdw=0.1662, w_hb=0.1209, w_el=0.1406, w_sol=0.1322, w_tor=0.2983,
    coulomb=332.06363,
    diel_A=-8.5525, diel_eps0=78.4, diel_lambda=0.003627, diel_k=7.7839,
    sigma=3.6, qasp=0.01097,
    smooth=0.5,        # smoothing band width for vdW / H-bond (A)
    cutoff=8.0,        # map cutoff for vdW / H-bond / desolvation (A)
    cap=1.0e5,         # cap on affinity-map node values (kcal/mol)
    r_floor=0.01,      # distance floor (A)
    k_out=1.0e3,       # out-of-grid restraint (kcal/mol/A^2)
)


def forcefield() -> dict:
    """The frozen parameter table as a plain dict of lists and floats."""
    ff = dict(FF_SCALARS)
    ff["n_types"] = len(TYPE_TABLE)
    ff["names"] = list(TYPE_NAMES)
    ff["Rii"] = [r[1] for r in TYPE_TABLE]
    ff["epsii"] = [r[2] for r in TYPE_TABLE]
    ff["vol"] = [r[3] for r in TYPE_TABLE]
    ff["solpar"] = [r[4] for r in TYPE_TABLE]
    ff["hbrole"] = [r[5] for r in TYPE_TABLE]
    ff["Rhb"] = [r[6] for r in TYPE_TABLE]
    ff["epshb"] = [r[7] for r in TYPE_TABLE]
    return ff


# Atom-type frequencies of the workloads (ligands and receptors).
FREQ_SIX = {"C": 0.55, "A": 0.15, "N": 0.10, "OA": 0.12, "HD": 0.05, "S": 0.03}
# Maximum bond count per type for the random trees.
MAX_VALENCE = {"C": 4, "A": 3, "N": 3, "NA": 3, "OA": 2, "S": 2, "SA": 2, "HD": 1}


# ---------------------------------------------------------------------------
# Grids
# ---------------------------------------------------------------------------
@dataclass
class Grid:
    n: tuple            # (nx, ny, nz)
    spacing: float
    origin: tuple       # coordinates of node (0,0,0)
    map_types: list     # force-field type id of each affinity map, in map order

    @property
    def extent(self):
        return tuple((k - 1) * self.spacing for k in self.n)

    @property
    def center(self):
        return tuple(o + e / 2 for o, e in zip(self.origin, self.extent))


def make_grid(n, spacing=0.375, center=(0.0, 0.0, 0.0), map_types=None) -> Grid:
    if isinstance(n, int):
        n = (n, n, n)
    if map_types is None:
        map_types = list(range(len(TYPE_TABLE)))
    origin = tuple(float(c - (k - 1) * spacing / 2) for c, k in zip(center, n))
    return Grid(tuple(int(k) for k in n), float(spacing), origin, list(map_types))


# ---------------------------------------------------------------------------
# Receptor
# ---------------------------------------------------------------------------
@dataclass
class Receptor:
    xyz: np.ndarray     # [n,3] float32
    types: np.ndarray   # [n] int32
    charges: np.ndarray  # [n] float32
    pocket: list = field(default_factory=list)  # [(center xyz, radius)]


def _draw_types(rng, n, freqs):
    names = list(freqs)
    p = np.array([freqs[k] for k in names], dtype=np.float64)
    p /= p.sum()
    idx = rng.choice(len(names), size=n, p=p)
    return np.array([TYPE_ID[names[i]] for i in idx], dtype=np.int32)


def _neutral_charges(rng, n, sd=0.2):
    q = rng.normal(0.0, sd, size=n)
    q -= q.mean()
    return q.astype(np.float32)


def receptor(seed: int, n_atoms: int, side: float | None = None,
             center=(0.0, 0.0, 0.0), n_pocket_spheres: int = 3,
             freqs=FREQ_SIX) -> Receptor:
    """Uniform atoms in a cube of side `side`, none inside a seeded pocket.

    The pocket is a union of spheres of radius U(5,7) A whose centres lie
    within 2.5 A of the cube centre.  Rejected atoms are redrawn, so the atom
    count is exact.  Default side: 20 A at 2,000 atoms, scaled as n^(1/3).
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    if side is None:
        side = 20.0 * (n_atoms / 2000.0) ** (1.0 / 3.0)
    c = np.asarray(center, dtype=np.float64)
    pocket = []
    for _ in range(n_pocket_spheres):
        off = rng.uniform(-2.5, 2.5, size=3)
        pocket.append((c + off, float(rng.uniform(5.0, 7.0))))
    out = np.empty((0, 3))
    while out.shape[0] < n_atoms:
        cand = c + rng.uniform(-side / 2, side / 2, size=(2 * n_atoms, 3))
        keep = np.ones(len(cand), dtype=bool)
        for pc, pr in pocket:
            keep &= np.linalg.norm(cand - pc, axis=1) >= pr
        out = np.concatenate([out, cand[keep]], axis=0)
    xyz = out[:n_atoms].astype(np.float32)
    types = _draw_types(rng, n_atoms, freqs)
    q = _neutral_charges(rng, n_atoms)
    return Receptor(xyz, types, q, [(tuple(p), r) for p, r in pocket])


# ---------------------------------------------------------------------------
# Ligands
# ---------------------------------------------------------------------------
@dataclass
class Ligand:
    types: np.ndarray      # [N] int32 force-field type ids
    charges: np.ndarray    # [N] float32
    xyz: np.ndarray        # [N,3] float32 reference conformation
    bonds: np.ndarray      # [N-1,2] int32
    rotatable: np.ndarray  # [N-1] uint8 (1 = rotatable)

    @property
    def n_atoms(self):
        return int(len(self.types))

    @property
    def n_torsions(self):
        return int(self.rotatable.sum())


def _tree_paths(n, bonds):
    adj = [[] for _ in range(n)]
    for a, b in bonds:
        adj[a].append(b)
        adj[b].append(a)
    dist = np.full((n, n), -1, dtype=np.int32)
    for s in range(n):
        dist[s, s] = 0
        stack = [s]
        while stack:
            u = stack.pop()
            for v in adj[u]:
                if dist[s, v] < 0:
                    dist[s, v] = dist[s, u] + 1
                    stack.append(v)
    return adj, dist


def _unit(v):
    return v / np.linalg.norm(v)


def _place(rng, x, parent_of, p, blen, placed, pathd, min_nonlocal, tries):
    """Try to place a new atom bonded to p; returns coordinates or None.

    Bond angle to p's parent 109.5 +- 5 degrees with a random dihedral (random
    direction when p is the first atom).  Pairs at bond-path distance 2 must be
    >= 1.2 A apart and pairs at distance >= 3 at least `min_nonlocal` A.
    """
    gp = parent_of[p]
    for _ in range(tries):
        if gp < 0:
            d = _unit(rng.normal(size=3))
        else:
            ang = math.radians(109.5 + rng.uniform(-5.0, 5.0))
            b = _unit(x[gp] - x[p])
            h = _unit(np.cross(b, rng.normal(size=3)))
            phi = rng.uniform(-math.pi, math.pi)
            perp = h * math.cos(phi) + np.cross(b, h) * math.sin(phi)
            d = b * math.cos(ang) + perp * math.sin(ang)
        cand = x[p] + blen * d
        ok = True
        for j in placed:
            dj = pathd[p][j] + 1
            r = float(np.linalg.norm(cand - x[j]))
            if (dj >= 3 and r < min_nonlocal) or (dj == 2 and r < 1.2):
                ok = False
                break
        if ok:
            return cand
    return None


def ligand(seed: int, n_atoms: int, n_torsions: int, freqs=FREQ_SIX,
           shuffle: bool = False, min_nonlocal: float = 2.0) -> Ligand:
    """Random typed tree ligand with a clash-free reference conformation.

    Topology and geometry grow together: each new heavy atom picks a random
    parent with free valence (per-type caps) and a bond length U(1.0, 1.55) A;
    parents without room for a clash-free placement are skipped (a molecule
    that cannot grow is redrawn from the next seed state).  HD atoms are
    leaves on N or OA (a C leaf replaces an HD that finds no host).  Rotatable
    bonds are drawn uniformly from the bonds whose two atoms both have degree
    >= 2; T = min(n_torsions, eligible).  Charges ~ N(0, 0.2), shifted to sum to
    zero.  With shuffle=True atom indices, bond order and bond direction are
    randomly permuted (same molecule).
    """
    assert n_atoms >= 1
    rng = np.random.default_rng(np.random.PCG64(seed))
    for _attempt in range(100):
        lig = _grow(rng, n_atoms, n_torsions, freqs, min_nonlocal)
        if lig is not None:
            break
    else:
        raise RuntimeError("ligand generator could not embed %d atoms" % n_atoms)
    if shuffle:
        lig = permute(lig, rng.permutation(n_atoms), rng.permutation(len(lig.bonds)), rng)
    return lig


def _grow(rng, n_atoms, n_torsions, freqs, min_nonlocal):
    hd_frac = freqs.get("HD", 0.0)
    heavy_freqs = {k: v for k, v in freqs.items() if k != "HD"}
    n_hd = int(rng.binomial(n_atoms, hd_frac)) if n_atoms >= 3 else 0
    n_heavy = n_atoms - n_hd
    types = list(_draw_types(rng, n_heavy, heavy_freqs))
    kinds = types + [TYPE_ID["HD"]] * n_hd
    x = np.zeros((n_atoms, 3))
    parent_of = [-1]
    deg = [0]
    pathd = [[0]]          # pathd[i][j]: bond-path distance between placed atoms
    placed = [0]
    out_types = [kinds[0]]
    for i in range(1, n_atoms):
        want = kinds[i]
        if want == TYPE_ID["HD"]:
            hosts = [j for j in placed if TYPE_NAMES[out_types[j]] in ("N", "OA")
                     and deg[j] < MAX_VALENCE[TYPE_NAMES[out_types[j]]]]
            if not hosts:
                want = TYPE_ID["C"]
        if want != TYPE_ID["HD"]:
            hosts = [j for j in placed if deg[j] < MAX_VALENCE[TYPE_NAMES[out_types[j]]]]
        order = list(rng.permutation(len(hosts)))
        pos = None
        for k in order:
            p = hosts[k]
            pos = _place(rng, x, parent_of, p, rng.uniform(1.0, 1.55), placed, pathd,
                         min_nonlocal, tries=24)
            if pos is not None:
                break
        if pos is None:
            return None
        x[i] = pos
        parent_of.append(p)
        deg.append(1)
        deg[p] += 1
        for j in placed:
            pathd[j].append(pathd[j][p] + 1)
        pathd.append([pathd[p][j] + 1 for j in placed] + [0])
        placed.append(i)
        out_types.append(want)
    n = n_atoms
    bonds = np.array([(parent_of[i], i) for i in range(1, n)], dtype=np.int32).reshape(-1, 2)
    degree = np.bincount(bonds.ravel(), minlength=n) if n > 1 else np.zeros(1, int)
    eligible = [b for b in range(len(bonds)) if degree[bonds[b, 0]] >= 2 and degree[bonds[b, 1]] >= 2]
    t = min(n_torsions, len(eligible))
    rot = np.zeros(len(bonds), dtype=np.uint8)
    if t > 0:
        pick = rng.choice(len(eligible), size=t, replace=False)
        rot[[eligible[k] for k in pick]] = 1
    q = _neutral_charges(rng, n)
    x = x - x.mean(axis=0)
    return Ligand(np.array(out_types, dtype=np.int32), q, x.astype(np.float32), bonds, rot)


def permute(lig: Ligand, atom_perm, bond_perm=None, rng=None) -> Ligand:
    """Relabel atoms: new atom k is old atom atom_perm[k]; bonds reordered by
    bond_perm and each bond's endpoint order optionally flipped."""
    atom_perm = np.asarray(atom_perm)
    n = len(atom_perm)
    inv = np.empty(n, dtype=np.int64)
    inv[atom_perm] = np.arange(n)
    bonds = inv[lig.bonds]
    rot = lig.rotatable.copy()
    if bond_perm is not None:
        bonds = bonds[bond_perm]
        rot = rot[bond_perm]
    if rng is not None and len(bonds):
        flip = rng.random(len(bonds)) < 0.5
        bonds[flip] = bonds[flip][:, ::-1]
    return Ligand(lig.types[atom_perm].copy(), lig.charges[atom_perm].copy(),
                  lig.xyz[atom_perm].copy(), bonds.astype(np.int32), rot.astype(np.uint8))


def lognormal_atoms(rng, median=32, sigma=0.4, lo=10, hi=100):
    return int(np.clip(round(median * math.exp(rng.normal(0.0, sigma))), lo, hi))


def ligand_set(seed: int, n_ligands: int, atoms=(15, 60), torsions=(0, 15),
               dist="uniform", freqs=FREQ_SIX) -> list:
    """A list of ligands.  dist='uniform': N ~ U[atoms], T ~ U[torsions];
    dist='lognormal': N lognormal (median 32, sigma 0.4, clipped to atoms)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    out = []
    for k in range(n_ligands):
        if dist == "uniform":
            n = int(rng.integers(atoms[0], atoms[1] + 1))
        else:
            n = lognormal_atoms(rng, lo=atoms[0], hi=atoms[1])
        t = int(rng.integers(torsions[0], torsions[1] + 1))
        out.append(ligand(int(rng.integers(1 << 62)), n, t, freqs=freqs))
    return out


# ---------------------------------------------------------------------------
# Fast C generator for large ligand sets (same recipe, its own random stream)
# ---------------------------------------------------------------------------
_LIGEN_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ligen.c")
_LIGEN_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libligen.so")
_ligen = None


def build_ligen() -> str:
    """Compile synth/ligen.c (gcc -O2 -fopenmp) into synth/libligen.so."""
    tmp = _LIGEN_LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _LIGEN_SRC, "-o", tmp, "-lm"], check=True,
                   capture_output=True)
    os.replace(tmp, _LIGEN_LIB)
    return _LIGEN_LIB


def _ligen_lib():
    global _ligen
    if _ligen is None:
        if not os.path.exists(_LIGEN_LIB) or os.path.getmtime(_LIGEN_LIB) < os.path.getmtime(_LIGEN_SRC):
            build_ligen()
        L = ctypes.CDLL(_LIGEN_LIB)
        vp = ctypes.c_void_p
        L.lg_ligand_set.argtypes = [ctypes.c_uint64, ctypes.c_int, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp, vp]
        L.lg_ligand_set.restype = ctypes.c_int
        _ligen = L
    return _ligen


@dataclass
class LigandPack:
    """Ligands stored back to back: ligand i owns n_atoms_per_ligand[i] atoms
    and n_bonds_per_ligand[i] bonds, in order."""
    n_atoms_per_ligand: np.ndarray   # [n] int32
    n_bonds_per_ligand: np.ndarray   # [n] int32
    types: np.ndarray                # [sum atoms] int32
    charges: np.ndarray              # [sum atoms] float32
    xyz: np.ndarray                  # [sum atoms, 3] float32
    bonds: np.ndarray                # [sum bonds, 2] int32 (indices local to the ligand)
    rotatable: np.ndarray            # [sum bonds] uint8

    def __len__(self):
        return len(self.n_atoms_per_ligand)

    def __getitem__(self, i) -> Ligand:
        if not -len(self) <= i < len(self):
            raise IndexError(i)
        return self.ligands([i % len(self)])[0]

    def __iter__(self):
        return iter(self.ligands())

    def ligands(self, idx=None) -> list:
        """Ligand objects (views) for the given indices (default: all)."""
        ao = np.concatenate([[0], np.cumsum(self.n_atoms_per_ligand)])
        bo = np.concatenate([[0], np.cumsum(self.n_bonds_per_ligand)])
        sel = range(len(self)) if idx is None else idx
        return [Ligand(self.types[ao[i]:ao[i + 1]], self.charges[ao[i]:ao[i + 1]], self.xyz[ao[i]:ao[i + 1]],
                       self.bonds[bo[i]:bo[i + 1]], self.rotatable[bo[i]:bo[i + 1]]) for i in sel]

    def subset(self, idx) -> "LigandPack":
        return pack_ligands(self.ligands(idx))


def pack_ligands(ligs) -> LigandPack:
    return LigandPack(np.array([l.n_atoms for l in ligs], np.int32), np.array([len(l.bonds) for l in ligs], np.int32),
                      np.concatenate([l.types for l in ligs]).astype(np.int32),
                      np.concatenate([l.charges for l in ligs]).astype(np.float32),
                      np.concatenate([l.xyz for l in ligs]).astype(np.float32),
                      np.concatenate([np.asarray(l.bonds).reshape(-1, 2) for l in ligs]).astype(np.int32),
                      np.concatenate([l.rotatable for l in ligs]).astype(np.uint8))


def ligand_set_fast(seed: int, n_ligands: int, atoms=(10, 100), torsions=(0, 32), dist="lognormal",
                    freqs=FREQ_SIX, min_nonlocal: float = 2.0, packed: bool = False):
    """Like ligand_set, generated by the C generator (about 10^5 ligands/s on
    8 cores).  Sizes and torsion requests are drawn here with numpy from
    `seed`; ligand i is grown from seed * 2^20 + i.  packed=True returns a
    LigandPack (the same ligands back to back) instead of a list."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    if dist == "uniform":
        n = rng.integers(atoms[0], atoms[1] + 1, size=n_ligands)
    else:
        n = np.array([lognormal_atoms(rng, lo=atoms[0], hi=atoms[1]) for _ in range(n_ligands)])
    t = rng.integers(torsions[0], torsions[1] + 1, size=n_ligands)
    n = np.ascontiguousarray(n, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    fr = np.zeros(len(TYPE_TABLE), dtype=np.float64)
    for k, v in freqs.items():
        fr[TYPE_ID[k]] = v
    na = int(n.sum())
    nb = int(np.maximum(n - 1, 0).sum())
    types = np.empty(na, np.int32)
    q = np.empty(na, np.float32)
    xyz = np.empty((na, 3), np.float32)
    bonds = np.empty((max(nb, 1), 2), np.int32)
    rot = np.empty(max(nb, 1), np.uint8)
    rc = _ligen_lib().lg_ligand_set((seed << 20) & (2**64 - 1), n_ligands, n.ctypes.data, t.ctypes.data,
                                    fr.ctypes.data, min_nonlocal, types.ctypes.data, q.ctypes.data,
                                    xyz.ctypes.data, bonds.ctypes.data, rot.ctypes.data)
    if rc:
        raise RuntimeError(f"C ligand generator failed on ligand {-rc - 1}")
    if packed:
        return LigandPack(n, np.maximum(n - 1, 0).astype(np.int32), types, q, xyz, bonds[:nb], rot[:nb])
    out = []
    a = b = 0
    for i in range(n_ligands):
        k = int(n[i])
        out.append(Ligand(types[a:a + k], q[a:a + k], xyz[a:a + k], bonds[b:b + k - 1], rot[b:b + k - 1]))
        a += k
        b += k - 1
    return out


# ---------------------------------------------------------------------------
# Genotypes  [t(3) | q(4: w,x,y,z) | theta(T)], stride 40
# ---------------------------------------------------------------------------
GENO_STRIDE = 40


def random_genotypes(seed: int, n: int, n_torsions, grid: Grid, margin: float = 0.0,
                     normalize_q: bool = False, outside_frac: float = 0.0) -> np.ndarray:
    """Random poses: t uniform in the grid box shrunk by `margin` (a fraction
    `outside_frac` are placed up to 3 A outside the box), q a random 4-vector
    (unit if normalize_q), theta uniform in (-pi, pi].  n_torsions may be an
    int or a per-pose array; unused slots are zero."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    g = np.zeros((n, GENO_STRIDE), dtype=np.float32)
    lo = np.array(grid.origin) + margin
    hi = np.array(grid.origin) + np.array(grid.extent) - margin
    t = rng.uniform(lo, hi, size=(n, 3))
    if outside_frac > 0:
        out = rng.random(n) < outside_frac
        t[out] = rng.uniform(lo - 3.0, hi + 3.0, size=(int(out.sum()), 3))
    g[:, 0:3] = t
    q = rng.normal(size=(n, 4))
    if normalize_q:
        q /= np.linalg.norm(q, axis=1, keepdims=True)
    else:
        q *= rng.uniform(0.5, 2.0, size=(n, 1))
    g[:, 3:7] = q
    nt = np.broadcast_to(np.asarray(n_torsions), (n,))
    th = rng.uniform(-math.pi, math.pi, size=(n, 32))
    for i in range(n):
        g[i, 7:7 + nt[i]] = th[i, :nt[i]]
    return g


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------
SIX_TYPES = [TYPE_ID[k] for k in ("C", "A", "N", "OA", "HD", "S")]
ALL_TYPES = list(range(len(TYPE_TABLE)))


def config(name: str, seed: int = 20200707, n_ligands: int | None = None) -> dict:
    """Synthetic stand-ins for the paper-scale workloads.

    single24:  1 ligand, N=24, T=5; 2,000-atom receptor in a 20 A cube; 40^3 grid, 6 type maps.
    screen64:  64 ligands, N~U[15,60], T~U[0,15]; 8,000-atom receptor; 64^3 grid, 8 type maps.
    batch4096: 4,096 ligands, N lognormal (median 32) in [10,100], T~U[0,32]; 80^3 grid
               (ligands from the C generator, as a LigandPack).
    campaign:  ligands as batch4096 on a 126^3 grid.
    """
    if name == "single24":
        rec = receptor(seed, 2000, side=20.0)
        grid = make_grid(40, 0.375, map_types=SIX_TYPES)
        ligs = [ligand(seed + 1, 24, 5)]
        dock = dict(nrun=4, pop=50, max_gens=50, max_evals=10**9, ls_rate=0.06, ls_iters=300)
    elif name == "screen64":
        rec = receptor(seed, 8000)
        grid = make_grid(64, 0.375, map_types=ALL_TYPES)
        ligs = ligand_set(seed + 1, n_ligands or 64, atoms=(15, 60), torsions=(0, 15))
        dock = dict(nrun=20, pop=150, max_gens=10**9, max_evals=2_500_000, ls_rate=0.06, ls_iters=300)
    elif name == "batch4096":
        rec = receptor(seed, 8000)
        grid = make_grid(80, 0.375, map_types=ALL_TYPES)
        ligs = ligand_set_fast(seed + 1, n_ligands or 4096, atoms=(10, 100), torsions=(0, 32),
                               dist="lognormal", packed=True)
        dock = dict(nrun=10, pop=150, max_gens=10**9, max_evals=100_000, ls_rate=0.06, ls_iters=300)
    elif name == "campaign":
        rec = receptor(seed, 8000)
        grid = make_grid(126, 0.375, map_types=ALL_TYPES)
        ligs = ligand_set_fast(seed + 1, n_ligands or 65536, atoms=(10, 100), torsions=(0, 32),
                               dist="lognormal", packed=True)
        dock = dict(nrun=20, pop=150, max_gens=10**9, max_evals=2_500_000, ls_rate=0.06, ls_iters=300)
    else:
        raise KeyError(name)
    return dict(name=name, receptor=rec, grid=grid, ligands=ligs, dock=dock, seed=seed)
