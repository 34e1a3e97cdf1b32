"""ctypes binding of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It loads ``liboracle.so`` (plain C, built from ``oracle.c`` with
gcc) and never touches the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
COUNT_LIB_PATH = os.path.join(HERE, "liboracle_opcount.so")
MAXT, MAXA, MAXTOR, STRIDE = 16, 128, 32, 40


def build(verbose: bool = False) -> str:
    """Compile liboracle.so and its op-counting build liboracle_opcount.so
    (oracle.c compiled as C++ with a counting double, opcount.hpp); always
    recompiles."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-parameter",
           os.path.join(HERE, "oracle.c"), "-o", LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-I", HERE,
           os.path.join(HERE, "opcount.cpp"), "-o", COUNT_LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(COUNT_LIB_PATH + ".tmp", COUNT_LIB_PATH)
    return LIB_PATH


class FF(C.Structure):
    _fields_ = [("n_types", C.c_int)] + [
        (k, C.c_double * MAXT) for k in ("Rii", "epsii", "vol", "solpar", "Rhb", "epshb")
    ] + [("hbrole", C.c_int * MAXT)] + [
        (k, C.c_double) for k in ("w_vdw", "w_hb", "w_el", "w_sol", "w_tor", "coulomb", "diel_A",
                                  "diel_eps0", "diel_lambda", "diel_k", "sigma", "qasp", "smooth",
                                  "cutoff", "cap", "r_floor", "k_out")
    ]


class DockParams(C.Structure):
    _fields_ = [("nrun", C.c_int), ("pop", C.c_int), ("max_gens", C.c_int), ("max_evals", C.c_int64),
                ("ls_rate", C.c_double), ("ls_iters", C.c_int), ("cx_rate", C.c_double),
                ("mut_rate", C.c_double), ("tour_p", C.c_double), ("rho", C.c_double),
                ("eps", C.c_double), ("mut_t", C.c_double), ("mut_theta", C.c_double),
                ("mut_rot", C.c_double), ("ls_method", C.c_int), ("autostop", C.c_int),
                ("sw_rho", C.c_double), ("sw_rho_lb", C.c_double), ("sw_max_succ", C.c_int),
                ("sw_max_fail", C.c_int), ("sw_sigma_t", C.c_double), ("sw_sigma_ang", C.c_double),
                ("stop_std", C.c_double)]


DEFAULT_DOCK = dict(nrun=4, pop=50, max_gens=50, max_evals=10**12, ls_rate=0.06, ls_iters=300,
                    cx_rate=0.8, mut_rate=0.02, tour_p=0.6, rho=0.8, eps=1e-2, mut_t=2.0,
                    mut_theta=np.pi / 2, mut_rot=np.pi / 2, ls_method=0, autostop=0,
                    sw_rho=1.0, sw_rho_lb=0.01, sw_max_succ=4, sw_max_fail=4, sw_sigma_t=1.0,
                    sw_sigma_ang=0.2, stop_std=0.15)


def make_ff(ff: dict) -> FF:
    s = FF()
    s.n_types = ff["n_types"]
    for k in ("Rii", "epsii", "vol", "solpar", "Rhb", "epshb", "hbrole"):
        arr = getattr(s, k)
        for i, v in enumerate(ff[k]):
            arr[i] = v
    for k in ("w_vdw", "w_hb", "w_el", "w_sol", "w_tor", "coulomb", "diel_A", "diel_eps0",
              "diel_lambda", "diel_k", "sigma", "qasp", "smooth", "cutoff", "cap", "r_floor", "k_out"):
        setattr(s, k, float(ff[k]))
    return s


def make_params(**kw) -> DockParams:
    d = dict(DEFAULT_DOCK)
    d.update({k: v for k, v in kw.items() if k in d})
    p = DockParams()
    for k, v in d.items():
        setattr(p, k, v)
    return p


_libs = {}


def lib(counting: bool = False):
    """The oracle library; counting=True: its op-counting build (same C ABI
    plus orc_opcount_reset / orc_opcount_get)."""
    if counting not in _libs:
        path = COUNT_LIB_PATH if counting else LIB_PATH
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        vp, ip, dp, fp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_float)
        u32 = C.c_uint32
        L.orc_philox4x32_10.argtypes = [C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
        L.orc_stream_word.argtypes = [C.c_uint64, u32, u32, u32, u32, u32, u32]
        L.orc_stream_word.restype = u32
        for name in ("orc_lj",):
            getattr(L, name).argtypes = [C.POINTER(FF), C.c_int, C.c_int, C.c_double, dp]
            getattr(L, name).restype = C.c_double
        L.orc_diel.argtypes = [C.POINTER(FF), C.c_double, dp]
        L.orc_diel.restype = C.c_double
        L.orc_elec.argtypes = [C.POINTER(FF), C.c_double, C.c_double, C.c_double, dp]
        L.orc_elec.restype = C.c_double
        for name in ("orc_desolv", "orc_pair"):
            getattr(L, name).argtypes = [C.POINTER(FF), C.c_int, C.c_double, C.c_int, C.c_double, C.c_double, dp]
            getattr(L, name).restype = C.c_double
        L.orc_grid_create.argtypes = [C.POINTER(FF), ip, C.c_double, dp, C.c_int, ip, fp]
        L.orc_grid_create.restype = vp
        L.orc_grid_set_receptor.argtypes = [vp, C.c_int, fp, ip, fp, C.c_int]
        L.orc_grid_node.argtypes = [vp, C.c_int, C.c_int, C.c_int, fp]
        L.orc_grid_values.argtypes = [vp]
        L.orc_grid_values.restype = fp
        L.orc_grid_free.argtypes = [vp]
        L.orc_node_values.argtypes = [vp, C.c_int, C.c_int, C.c_int, dp]
        L.orc_ligand_new.restype = vp
        L.orc_ligand_free.argtypes = [vp]
        L.orc_ligand_prepare.argtypes = [vp, C.POINTER(FF), C.c_int, C.c_int, ip, C.POINTER(C.c_ubyte),
                                         ip, fp, fp]
        L.orc_ligand_msg.argtypes = [vp]
        L.orc_ligand_msg.restype = C.c_char_p
        L.orc_ligand_info.argtypes = [vp, ip]
        L.orc_ligand_pairs.argtypes = [vp, ip, ip]
        L.orc_ligand_torsion.argtypes = [vp, C.c_int, ip, ip, ip, C.POINTER(C.c_ubyte)]
        L.orc_pose.argtypes = [vp, dp, C.c_int, dp]
        L.orc_score.argtypes = [vp, vp, dp, dp, dp, dp, dp]
        L.orc_score_batch.argtypes = [C.POINTER(vp), ip, C.c_int, vp, fp, dp, dp, dp, C.c_int]
        L.orc_max_threads.restype = C.c_int
        L.orc_genotype_rotate.argtypes = [dp, dp]
        L.orc_init_individual.argtypes = [vp, vp, C.c_uint64, u32, u32, u32, dp]
        L.orc_ga_offspring.argtypes = [vp, C.POINTER(DockParams), C.c_uint64, u32, u32, u32, C.c_int,
                                       dp, dp, dp, dp]
        L.orc_ls_pick.argtypes = [C.c_uint64, u32, u32, u32, C.c_int, C.c_int, ip]
        L.orc_adadelta.argtypes = [vp, vp, C.POINTER(DockParams), dp, C.c_int, dp, dp]
        L.orc_n_ls.argtypes = [C.POINTER(DockParams)]
        L.orc_solis_wets.argtypes = [vp, vp, C.POINTER(DockParams), dp, C.c_double, C.c_int, C.c_uint64, u32, u32,
                                     u32, u32, dp, dp, ip]
        L.orc_sw_deviate.argtypes = [C.c_uint64, u32, u32, u32, u32, u32, C.c_int]
        L.orc_sw_deviate.restype = C.c_double
        L.orc_dock_run.argtypes = [vp, vp, C.POINTER(DockParams), C.c_uint64, u32, u32, dp, dp,
                                   C.POINTER(C.c_int64), ip]
        L.orc_dock.argtypes = [vp, vp, C.POINTER(DockParams), C.c_uint64, u32, dp, dp,
                               C.POINTER(C.c_int64), ip, C.c_int]
        if counting:
            L.orc_opcount_reset.argtypes = []
            L.orc_opcount_reset.restype = None
            L.orc_opcount_get.argtypes = [C.POINTER(C.c_uint64)]
            L.orc_opcount_get.restype = None
        _libs[counting] = L
    return _libs[counting]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# pair functions
# --------------------------------------------------------------------------
class Oracle:
    """Thin object holding the force field; all methods call the C oracle."""

    def __init__(self, ff: dict, counting: bool = False):
        self.ff_dict = ff
        self.ff = make_ff(ff)
        self.L = lib(counting)
        self.counting = counting

    def opcount(self, fn, *args, **kw):
        """(fn's result, floating-point operations it ran) with the op-counting
        build: {add, mul, div, func, total}; add counts subtractions, func the
        transcendentals (each one operation)."""
        assert self.counting, "needs Oracle(ff, counting=True)"
        self.L.orc_opcount_reset()
        out = fn(*args, **kw)
        c = (C.c_uint64 * 4)()
        self.L.orc_opcount_get(c)
        d = dict(add=int(c[0]), mul=int(c[1]), div=int(c[2]), func=int(c[3]))
        d["total"] = sum(d.values())
        return out, d

    # pair terms -----------------------------------------------------------
    def lj(self, ti, tj, r):
        d = C.c_double()
        e = self.L.orc_lj(C.byref(self.ff), ti, tj, r, C.byref(d))
        return e, d.value

    def diel(self, r):
        d = C.c_double()
        e = self.L.orc_diel(C.byref(self.ff), r, C.byref(d))
        return e, d.value

    def elec(self, qi, qj, r):
        d = C.c_double()
        e = self.L.orc_elec(C.byref(self.ff), qi, qj, r, C.byref(d))
        return e, d.value

    def desolv(self, ti, qi, tj, qj, r):
        d = C.c_double()
        e = self.L.orc_desolv(C.byref(self.ff), ti, qi, tj, qj, r, C.byref(d))
        return e, d.value

    def pair(self, ti, qi, tj, qj, r):
        d = C.c_double()
        e = self.L.orc_pair(C.byref(self.ff), ti, qi, tj, qj, r, C.byref(d))
        return e, d.value

    # grids ----------------------------------------------------------------
    def grid(self, grid, receptor=None, values=None, lazy=False):
        return OracleGrid(self, grid, receptor, values, lazy)

    # ligands --------------------------------------------------------------
    def ligand(self, lig):
        return OracleLigand(self, lig)

    # philox ---------------------------------------------------------------
    def philox(self, ctr, key):
        c = (C.c_uint32 * 4)(*ctr)
        k = (C.c_uint32 * 2)(*key)
        o = (C.c_uint32 * 4)()
        self.L.orc_philox4x32_10(c, k, o)
        return [int(v) for v in o]

    def stream_word(self, seed, lig, run, gen, indiv, stream, w):
        return int(self.L.orc_stream_word(seed, lig, run, gen, indiv, stream, w))

    # scoring --------------------------------------------------------------
    def score(self, L, G, geno, want_xyz=False):
        g = np.zeros(STRIDE)
        g[:len(geno)] = np.asarray(geno, dtype=np.float64)[:STRIDE]
        E = C.c_double()
        grad = np.zeros(STRIDE)
        terms = np.zeros(3)
        xyz = np.zeros((L.n, 3))
        rc = self.L.orc_score(L.h, G.h, _p(g, C.c_double), C.byref(E), _p(grad, C.c_double),
                              _p(terms, C.c_double), _p(xyz, C.c_double))
        if rc:
            raise ValueError("oracle score failed (%d)" % rc)
        if want_xyz:
            return E.value, grad, terms, xyz
        return E.value, grad, terms

    def score_batch(self, ligs, lig_idx, G, genos, threads=0, grad=True):
        genos = _f32(genos)
        n = genos.shape[0]
        handles = (C.c_void_p * len(ligs))(*[l.h for l in ligs])
        idx = _i32(lig_idx)
        E = np.zeros(n)
        gr = np.zeros((n, STRIDE)) if grad else None
        terms = np.zeros((n, 3))
        rc = self.L.orc_score_batch(handles, _p(idx, C.c_int), n, G.h, _p(genos, C.c_float),
                                    _p(E, C.c_double), _p(gr, C.c_double) if grad else None,
                                    _p(terms, C.c_double), threads)
        if rc:
            raise ValueError("oracle batch score failed (%d)" % rc)
        return E, gr, terms

    def pose(self, L, geno, order=0):
        g = np.zeros(STRIDE)
        g[:len(geno)] = np.asarray(geno, dtype=np.float64)[:STRIDE]
        xyz = np.zeros((L.n, 3))
        self.L.orc_pose(L.h, _p(g, C.c_double), order, _p(xyz, C.c_double))
        return xyz

    def rotate(self, geno, w):
        g = _f64(geno).copy()
        ww = _f64(w)
        self.L.orc_genotype_rotate(_p(g, C.c_double), _p(ww, C.c_double))
        return g

    def max_threads(self):
        return int(self.L.orc_max_threads())

    # docking --------------------------------------------------------------
    def init_individual(self, L, G, seed, lig, run, indiv):
        g = np.zeros(STRIDE)
        self.L.orc_init_individual(L.h, G.h, seed, lig, run, indiv, _p(g, C.c_double))
        return g

    def ga_offspring(self, L, params, seed, lig, run, gen, old_geno, old_E):
        old_geno = _f64(old_geno)
        old_E = _f64(old_E)
        pop = old_E.shape[0]
        new_geno = np.zeros((pop, STRIDE))
        new_E = np.zeros(pop)
        self.L.orc_ga_offspring(L.h, C.byref(params), seed, lig, run, gen, pop, _p(old_geno, C.c_double),
                                _p(old_E, C.c_double), _p(new_geno, C.c_double), _p(new_E, C.c_double))
        return new_geno, new_E

    def ls_pick(self, seed, lig, run, gen, pop, n_ls):
        out = np.zeros(max(n_ls, 1), dtype=np.int32)
        self.L.orc_ls_pick(seed, lig, run, gen, pop, n_ls, _p(out, C.c_int))
        return out[:n_ls]

    def adadelta(self, L, G, params, geno, iters):
        g = np.zeros(STRIDE)
        g[:len(geno)] = np.asarray(geno, dtype=np.float64)[:STRIDE]
        best = np.zeros(STRIDE)
        E = C.c_double()
        rc = self.L.orc_adadelta(L.h, G.h, C.byref(params), _p(g, C.c_double), iters, _p(best, C.c_double),
                                 C.byref(E))
        if rc:
            raise ValueError("oracle adadelta failed (%d)" % rc)
        return best, E.value

    def solis_wets(self, L, G, params, geno, max_ev, seed, lig, run, gen, indiv, E_in=float("nan")):
        """Returns (best genotype, its energy, evaluations used)."""
        g = np.zeros(STRIDE)
        g[:len(geno)] = np.asarray(geno, dtype=np.float64)[:STRIDE]
        best = np.zeros(STRIDE)
        E = C.c_double()
        used = C.c_int()
        rc = self.L.orc_solis_wets(L.h, G.h, C.byref(params), _p(g, C.c_double), E_in, max_ev, seed, lig, run, gen,
                                   indiv, _p(best, C.c_double), C.byref(E), C.byref(used))
        if rc:
            raise ValueError("oracle solis-wets failed (%d)" % rc)
        return best, E.value, used.value

    def sw_deviate(self, seed, lig, run, gen, indiv, it, k):
        return float(self.L.orc_sw_deviate(seed, lig, run, gen, indiv, it, k))

    def n_ls(self, params):
        return int(self.L.orc_n_ls(C.byref(params)))

    def dock(self, L, G, params, seed, lig_id, threads=0):
        nrun = params.nrun
        geno = np.zeros((nrun, STRIDE))
        E = np.zeros(nrun)
        ev = np.zeros(nrun, dtype=np.int64)
        gens = np.zeros(nrun, dtype=np.int32)
        rc = self.L.orc_dock(L.h, G.h, C.byref(params), seed, lig_id, _p(geno, C.c_double), _p(E, C.c_double),
                             _p(ev, C.c_int64), _p(gens, C.c_int), threads)
        if rc:
            raise ValueError("oracle dock failed (%d)" % rc)
        return geno, E, ev, gens


class OracleGrid:
    def __init__(self, orc: Oracle, grid, receptor=None, values=None, lazy=False):
        self.o = orc
        self.grid = grid
        self.n_maps = len(grid.map_types)
        n = (C.c_int * 3)(*grid.n)
        origin = (C.c_double * 3)(*grid.origin)
        mt = (C.c_int * max(1, self.n_maps))(*grid.map_types)
        vals = None
        if values is not None:
            self._vals = _f32(values).reshape(-1)
            expect = (self.n_maps + 2) * grid.n[0] * grid.n[1] * grid.n[2]
            assert self._vals.size == expect, (self._vals.size, expect)
            vals = _p(self._vals, C.c_float)
        self.h = orc.L.orc_grid_create(C.byref(orc.ff), n, grid.spacing, origin, self.n_maps, mt, vals)
        if not self.h:
            raise ValueError("invalid grid")
        if receptor is not None:
            xyz = _f32(receptor.xyz)
            ty = _i32(receptor.types)
            q = _f32(receptor.charges)
            orc.L.orc_grid_set_receptor(self.h, len(ty), _p(xyz, C.c_float), _p(ty, C.c_int),
                                        _p(q, C.c_float), 1 if lazy else 0)

    def values(self):
        """Map values [n_maps+2, nz, ny, nx] (a copy)."""
        nx, ny, nz = self.grid.n
        ptr = self.o.L.orc_grid_values(self.h)
        a = np.ctypeslib.as_array(ptr, shape=((self.n_maps + 2) * nx * ny * nz,))
        return a.copy().reshape(self.n_maps + 2, nz, ny, nx)

    def node(self, i, j, k):
        out = np.zeros(self.n_maps + 2, dtype=np.float32)
        self.o.L.orc_grid_node(self.h, i, j, k, _p(out, C.c_float))
        return out

    def node_exact(self, i, j, k):
        """Unrounded (double) sums at a node; needs a receptor."""
        out = np.zeros(self.n_maps + 2)
        self.o.L.orc_node_values(self.h, i, j, k, _p(out, C.c_double))
        return out

    def __del__(self):
        try:
            self.o.L.orc_grid_free(self.h)
        except Exception:
            pass


class OracleLigand:
    def __init__(self, orc: Oracle, lig):
        self.o = orc
        self.lig = lig
        self.h = orc.L.orc_ligand_new()
        n = lig.n_atoms
        bonds = _i32(lig.bonds).reshape(-1)
        rot = np.ascontiguousarray(lig.rotatable, dtype=np.uint8)
        ty = _i32(lig.types)
        q = _f32(lig.charges)
        xyz = _f32(lig.xyz)
        rc = orc.L.orc_ligand_prepare(self.h, C.byref(orc.ff), n, len(lig.bonds),
                                      _p(bonds, C.c_int) if bonds.size else None,
                                      _p(rot, C.c_ubyte) if rot.size else None, _p(ty, C.c_int),
                                      _p(q, C.c_float), _p(xyz, C.c_float))
        self.rc = rc
        if rc:
            self.msg = orc.L.orc_ligand_msg(self.h).decode()
            raise ValueError("oracle ligand rejected: " + self.msg)
        info = (C.c_int * 5)()
        orc.L.orc_ligand_info(self.h, info)
        self.n, self.n_tor, self.n_pairs, self.n_frag, self.root_atom = list(info)

    def pairs(self):
        pi = np.zeros(max(1, self.n_pairs), dtype=np.int32)
        pj = np.zeros(max(1, self.n_pairs), dtype=np.int32)
        self.o.L.orc_ligand_pairs(self.h, _p(pi, C.c_int), _p(pj, C.c_int))
        return list(zip(pi[:self.n_pairs].tolist(), pj[:self.n_pairs].tolist()))

    def torsion(self, k):
        a, b, d = C.c_int(), C.c_int(), C.c_int()
        mv = np.zeros(self.n, dtype=np.uint8)
        self.o.L.orc_ligand_torsion(self.h, k, C.byref(a), C.byref(b), C.byref(d), _p(mv, C.c_ubyte))
        return a.value, b.value, d.value, mv.astype(bool)

    def __del__(self):
        try:
            self.o.L.orc_ligand_free(self.h)
        except Exception:
            pass
