"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-side validation accepts / rejects ligands as
specified."""
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "addock.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(ad_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def pkg():
    import paper_2007_03678_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pkg.build()
    return pkg


def test_library_exports_every_declared_symbol(pkg):
    L = pkg.lib()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(pkg.EXPORTS) == names


def test_library_links_no_oracle(pkg):
    # the product library must not depend on the test oracle
    import subprocess
    out = subprocess.run(["readelf", "-d", pkg.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out


def test_create_rejects_bad_device(pkg):
    import ctypes as C
    L = pkg.lib()
    ff = pkg.make_forcefield(synth.forcefield())
    h = C.c_void_p()
    assert L.ad_create(C.byref(h), 4096, C.byref(ff), None) == pkg.AD_E_DEVICE
    assert not h.value


def test_create_rejects_bad_forcefield(pkg):
    import ctypes as C
    L = pkg.lib()
    d = synth.forcefield()
    d["sigma"] = -1.0
    ff = pkg.make_forcefield(d)
    h = C.c_void_p()
    assert L.ad_create(C.byref(h), 0, C.byref(ff), None) == pkg.AD_E_INVALID


def test_ligand_check_accepts_generated_ligands(pkg):
    for seed, n, t in [(1, 1, 0), (2, 2, 0), (3, 24, 5), (4, 100, 32), (5, 128, 20)]:
        rc, msg = pkg.ad_ligand_check(synth.ligand(seed, n, t, shuffle=True), 8)
        assert rc == 0, msg


@pytest.mark.parametrize("case", ["cycle", "disconnected", "terminal", "index", "selfloop", "type", "nan",
                                  "toomanytor", "toolarge"])
def test_ligand_check_rejects(pkg, case):
    lig = synth.ligand(1, 10, 2)
    b, r, n = lig.bonds.copy(), lig.rotatable.copy(), lig.n_atoms
    types, q, xyz = lig.types.copy(), lig.charges.copy(), lig.xyz.copy()
    if case == "cycle":
        b[0] = b[1]
    elif case == "disconnected":
        b, r = b[:-1], r[:-1]
    elif case == "terminal":
        leaf = [i for i in range(n) if np.sum(b == i) == 1][0]
        r[int(np.where((b == leaf).any(axis=1))[0][0])] = 1
    elif case == "index":
        b[2] = [0, n]
    elif case == "selfloop":
        b[2] = [3, 3]
    elif case == "type":
        types[0] = 8
    elif case == "nan":
        xyz[3, 1] = np.nan
    elif case == "toomanytor":
        big = synth.ligand(3, 100, 40)
        types, q, xyz, b = big.types, big.charges, big.xyz, big.bonds
        deg = np.bincount(b.ravel(), minlength=100)
        r = ((deg[b[:, 0]] >= 2) & (deg[b[:, 1]] >= 2)).astype(np.uint8)
    elif case == "toolarge":
        big = synth.ligand(2, 128, 3)
        types = np.concatenate([big.types, [0]]).astype(np.int32)
        q = np.concatenate([big.charges, [0]]).astype(np.float32)
        xyz = np.concatenate([big.xyz, [[9, 9, 9]]]).astype(np.float32)
        b = np.concatenate([big.bonds, [[0, 128]]]).astype(np.int32)
        r = np.concatenate([big.rotatable, [0]]).astype(np.uint8)
    rc, msg = pkg.ad_ligand_check(synth.Ligand(types, q, xyz, b, r), 8)
    assert rc == pkg.AD_E_INVALID and msg


def test_oracle_and_product_accept_the_same_ligands(pkg, orc):
    """Both independent preparations agree on validity for random topologies."""
    rng = np.random.default_rng(0)
    for s in range(30):
        lig = synth.ligand(100 + s, int(rng.integers(2, 40)), int(rng.integers(0, 10)))
        b, r = lig.bonds.copy(), lig.rotatable.copy()
        if s % 3 == 1 and len(r):
            r[:] = 1          # some bonds end in leaves -> both must reject
        l2 = synth.Ligand(lig.types, lig.charges, lig.xyz, b, r)
        rc, _ = pkg.ad_ligand_check(l2, 8)
        try:
            orc.ligand(l2)
            ok = True
        except ValueError:
            ok = False
        assert (rc == 0) == ok


def test_grid_check_rejects_index_overflow(pkg):
    # the kernels multiply (map * nz + k) by nx * ny in 24-bit products
    ok = synth.Grid((40, 40, 40), 0.375, (0.0, 0.0, 0.0), list(range(8)))
    assert pkg.ad_grid_check(ok, 8) == (0, "")
    thin = synth.Grid((2, 2, 1 << 22), 0.375, (0.0, 0.0, 0.0), list(range(8)))   # 8 * 2^22 = 2^25 rows
    rc, msg = pkg.ad_grid_check(thin, 8)
    assert rc == pkg.AD_E_INVALID and "n_maps*nz" in msg
    wide = synth.Grid((4096, 4096, 2), 0.375, (0.0, 0.0, 0.0), [0])   # nx * ny = 2^24
    assert pkg.ad_grid_check(wide, 8)[0] == pkg.AD_E_INVALID
    for bad in (synth.Grid((1, 40, 40), 0.375, (0, 0, 0), [0]), synth.Grid((40, 40, 40), 0.0, (0, 0, 0), [0]),
                synth.Grid((40, 40, 40), 0.375, (0, 0, 0), [0, 0]), synth.Grid((40, 40, 40), 0.375, (0, 0, 0), [9])):
        assert pkg.ad_grid_check(bad, 8)[0] == pkg.AD_E_INVALID


def test_noalloc_limit_matches_the_header(pkg):
    txt = open(os.path.join(ROOT, "include", "addock.h")).read()
    m = re.search(r"#define AD_NOALLOC_MAX_POSES (\d+)", txt)
    assert m and int(m.group(1)) == pkg.NOALLOC_MAX_POSES
