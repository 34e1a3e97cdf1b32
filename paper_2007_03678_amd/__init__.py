"""Python binding of libaddock (C ABI in include/addock.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Host arrays are numpy; device arrays are torch CUDA tensors (torch
provides device memory and streams).  The library must be built
(``build()``); loading fails loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import subprocess
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libaddock.so")
SOURCES = ["csrc/prep.cpp", "csrc/api.cpp", "csrc/dock.cpp", "csrc/kernels.hip", "csrc/prescreen.hip",
           "csrc/microbench.hip"]

AD_OK, AD_E_INVALID, AD_E_NOMAP, AD_E_OOM, AD_E_DEVICE, AD_E_STATE, AD_E_UNSUPPORTED, AD_E_HIP = 0, -1, -2, -3, -4, -5, -6, -7
ERR_NAMES = {0: "AD_OK", -1: "AD_E_INVALID", -2: "AD_E_NOMAP", -3: "AD_E_OOM", -4: "AD_E_DEVICE",
             -5: "AD_E_STATE", -6: "AD_E_UNSUPPORTED", -7: "AD_E_HIP"}
MAX_TYPES, STRIDE = 16, 40
SHAPE_AUTO, SHAPE_WAVE64, SHAPE_WAVE128, SHAPE_PACKED = 0, 1, 2, 3
NOALLOC_MAX_POSES = 4096   # AD_NOALLOC_MAX_POSES

EXPORTS = ["ad_create", "ad_destroy", "ad_last_error", "ad_set_stream", "ad_synchronize", "ad_load_grids",
           "ad_build_grids", "ad_grid_check", "ad_ligand_check", "ad_load_ligands", "ad_load_ligands_packed", "ad_free_batch", "ad_dock_stream", "ad_batch_info",
           "ad_score_poses", "ad_score_poses_shape", "ad_score_poses_noalloc", "ad_dock_batch", "ad_dock_select", "ad_local_search", "ad_local_search_shape", "ad_solis_wets", "ad_initial_population",
           "ad_set_kernel_timing", "ad_get_kernel_timing", "ad_set_schedule", "ad_get_schedule", "ad_set_launch_shape",
           "ad_get_launch_shape", "ad_set_work_queue", "ad_get_work_queue",
           "ad_set_chains", "ad_get_chains", "ad_microbench",
           "ad_prescreen_n_params", "ad_prescreen_create",
           "ad_prescreen_destroy", "ad_prescreen_set_params", "ad_prescreen_get_params", "ad_prescreen_set_scale",
           "ad_prescreen_get_scale", "ad_prescreen_predict", "ad_prescreen_grad", "ad_prescreen_train"]


def build(verbose: bool = False, arch: str = "gfx950") -> str:
    """Compile libaddock.so in-tree with hipcc for gfx950 (always recompiles)."""
    # -ffp-contract=on: a*b+c is fused only within one source expression, so
    # every instantiation of the evaluation (with or without the gradient)
    # rounds the energy the same way and a returned pose re-scores bitwise
    cmd = ["hipcc", f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
           "-Wno-unused-result", "-Wno-unused-value",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-o", LIB_PATH + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-4000:])
    if verbose:
        print(r.stderr)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class AddockError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class ForceField(C.Structure):
    _fields_ = [("n_types", C.c_int)] + [
        (k, C.c_double * MAX_TYPES) for k in ("Rii", "epsii", "vol", "solpar", "Rhb", "epshb")
    ] + [("hbrole", C.c_int * MAX_TYPES)] + [
        (k, C.c_double) for k in ("w_vdw", "w_hb", "w_el", "w_sol", "w_tor", "coulomb", "diel_A",
                                  "diel_eps0", "diel_lambda", "diel_k", "sigma", "qasp", "smooth",
                                  "cutoff", "cap", "r_floor", "k_out")]


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("spacing", C.c_double),
                ("origin", C.c_double * 3), ("n_maps", C.c_int), ("map_types", C.POINTER(C.c_int))]


class Ligand(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("n_bonds", C.c_int), ("type_id", C.POINTER(C.c_int)),
                ("charge", C.POINTER(C.c_float)), ("xyz", C.POINTER(C.c_float)),
                ("bonds", C.POINTER(C.c_int)), ("rotatable", C.POINTER(C.c_ubyte))]


class DockParams(C.Structure):
    _fields_ = [("nrun", C.c_int), ("pop", C.c_int), ("max_gens", C.c_int), ("max_evals", C.c_int64),
                ("ls_rate", C.c_double), ("ls_iters", C.c_int), ("cx_rate", C.c_double),
                ("mut_rate", C.c_double), ("tour_p", C.c_double), ("rho", C.c_double), ("eps", C.c_double),
                ("mut_t", C.c_double), ("mut_theta", C.c_double), ("mut_rot", C.c_double),
                ("ls_method", C.c_int), ("autostop", C.c_int), ("sw_rho", C.c_double), ("sw_rho_lb", C.c_double),
                ("sw_max_succ", C.c_int), ("sw_max_fail", C.c_int), ("sw_sigma_t", C.c_double),
                ("sw_sigma_ang", C.c_double), ("stop_std", C.c_double)]


class KernelTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 4), ("launches", C.c_int64 * 4), ("busy_ms", C.c_double * 4)]


KERNEL_KINDS = ("init", "ga", "ls", "score")


class PrescreenCfg(C.Structure):
    _fields_ = [("batch_size", C.c_int), ("lr", C.c_double), ("lam", C.c_double), ("tau", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double), ("label_max", C.c_double)]


DEFAULT_PRESCREEN = dict(batch_size=256, lr=1e-3, lam=1.0, tau=0.5, beta1=0.9, beta2=0.999, eps=1e-8,
                         label_max=float("inf"))


class DockResult(C.Structure):
    _fields_ = [("best_energy", C.c_float), ("best_score", C.c_float),
                ("best_genotype", C.c_float * STRIDE), ("best_run", C.c_int),
                ("generations", C.c_int), ("evals", C.c_int64)]


DEFAULT_DOCK = dict(nrun=4, pop=50, max_gens=50, max_evals=2**62, ls_rate=0.06, ls_iters=300, cx_rate=0.8,
                    mut_rate=0.02, tour_p=0.6, rho=0.8, eps=1e-2, mut_t=2.0, mut_theta=np.pi / 2,
                    mut_rot=np.pi / 2, ls_method=0, autostop=0, sw_rho=1.0, sw_rho_lb=0.01, sw_max_succ=4,
                    sw_max_fail=4, sw_sigma_t=1.0, sw_sigma_ang=0.2, stop_std=0.15)

_lib = None


def lib():
    """Load libaddock.so (torch first, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library will bind to)
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2007_03678_amd.build() first")
    L = C.CDLL(LIB_PATH)
    vp, ip, fp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_float)
    L.ad_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(ForceField), vp]
    L.ad_destroy.argtypes = [vp]
    L.ad_destroy.restype = None
    L.ad_last_error.argtypes = [vp]
    L.ad_last_error.restype = C.c_char_p
    L.ad_set_stream.argtypes = [vp, vp]
    L.ad_synchronize.argtypes = [vp]
    L.ad_load_grids.argtypes = [vp, C.POINTER(GridDesc), vp, C.c_int]
    L.ad_build_grids.argtypes = [vp, C.POINTER(GridDesc), C.c_int, fp, ip, fp, fp]
    L.ad_ligand_check.argtypes = [C.POINTER(Ligand), C.c_int, C.c_char_p, C.c_int]
    L.ad_grid_check.argtypes = [C.POINTER(GridDesc), C.c_int, C.c_char_p, C.c_int]
    L.ad_load_ligands.argtypes = [vp, C.c_int, C.POINTER(Ligand), C.POINTER(vp)]
    L.ad_load_ligands_packed.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp, C.POINTER(vp)]
    L.ad_dock_stream.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp, C.c_int, C.POINTER(DockParams),
                                 C.c_uint64, C.c_uint32, vp, C.POINTER(C.c_double)]
    L.ad_free_batch.argtypes = [vp]
    L.ad_free_batch.restype = None
    L.ad_batch_info.argtypes = [vp, C.c_int, ip, ip, ip, ip, ip]
    L.ad_set_kernel_timing.argtypes = [vp, C.c_int]
    L.ad_get_kernel_timing.argtypes = [vp, C.POINTER(KernelTimes), C.c_int]
    L.ad_score_poses.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp, C.c_int]
    L.ad_score_poses_shape.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp, C.c_int, C.c_int]
    L.ad_score_poses_noalloc.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp]
    L.ad_local_search_shape.argtypes = [vp, vp, C.c_int, vp, vp, vp, C.POINTER(DockParams), C.c_int, C.c_int,
                                        C.c_int]
    L.ad_dock_batch.argtypes = [vp, vp, C.POINTER(DockParams), C.c_uint64, vp, C.POINTER(DockResult), fp, fp]
    L.ad_dock_select.argtypes = [vp, vp, C.c_int, vp, C.POINTER(DockParams), C.c_uint64, C.POINTER(DockResult), fp,
                                 fp]
    L.ad_local_search.argtypes = [vp, vp, C.c_int, vp, vp, vp, C.POINTER(DockParams), C.c_int, C.c_int]
    L.ad_solis_wets.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, C.POINTER(DockParams), C.c_int, C.c_uint64]
    L.ad_initial_population.argtypes = [vp, vp, C.c_int, C.c_uint32, C.c_int, C.c_int, C.c_uint64, fp]
    L.ad_set_schedule.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
    L.ad_get_schedule.argtypes = [vp, ip, ip, ip]
    L.ad_set_launch_shape.argtypes = [vp, C.c_int, C.c_int]
    L.ad_get_launch_shape.argtypes = [vp, ip, ip]
    L.ad_set_work_queue.argtypes = [vp, C.c_int]
    L.ad_get_work_queue.argtypes = [vp, ip]
    L.ad_set_chains.argtypes = [vp, C.c_int]
    L.ad_microbench.argtypes = [vp, C.c_int, C.c_size_t, C.POINTER(C.c_double)]
    L.ad_get_chains.argtypes = [vp, ip]
    L.ad_prescreen_n_params.argtypes = []
    L.ad_prescreen_create.argtypes = [vp, C.POINTER(PrescreenCfg), C.c_uint64, C.POINTER(vp)]
    L.ad_prescreen_destroy.argtypes = [vp]
    L.ad_prescreen_destroy.restype = None
    L.ad_prescreen_set_params.argtypes = [vp, fp]
    L.ad_prescreen_get_params.argtypes = [vp, fp]
    L.ad_prescreen_set_scale.argtypes = [vp, C.c_double, C.c_double]
    L.ad_prescreen_get_scale.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.ad_prescreen_predict.argtypes = [vp, vp, C.c_int, vp, fp]
    L.ad_prescreen_grad.argtypes = [vp, vp, C.c_int, vp, fp, fp, fp, fp]
    L.ad_prescreen_train.argtypes = [vp, vp, C.c_int, vp, fp, C.c_int, C.c_uint64, fp]
    _lib = L
    return L


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def make_forcefield(ff: dict) -> ForceField:
    s = ForceField()
    s.n_types = ff["n_types"]
    for k in ("Rii", "epsii", "vol", "solpar", "Rhb", "epshb", "hbrole"):
        arr = getattr(s, k)
        for i, v in enumerate(ff[k]):
            arr[i] = v
    for k in ("w_vdw", "w_hb", "w_el", "w_sol", "w_tor", "coulomb", "diel_A", "diel_eps0", "diel_lambda",
              "diel_k", "sigma", "qasp", "smooth", "cutoff", "cap", "r_floor", "k_out"):
        setattr(s, k, float(ff[k]))
    return s


def make_params(**kw) -> DockParams:
    d = dict(DEFAULT_DOCK)
    for k, v in kw.items():
        if k in d:
            d[k] = v
    p = DockParams()
    for k, v in d.items():
        setattr(p, k, v)
    return p


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _is_device(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


class _LigandArrays:
    """Keeps numpy arrays alive while an ad_ligand points at them."""

    def __init__(self, lig):
        self.types = _np(lig.types, np.int32)
        self.q = _np(lig.charges, np.float32)
        self.xyz = _np(lig.xyz, np.float32).reshape(-1)
        self.bonds = _np(lig.bonds, np.int32).reshape(-1)
        self.rot = _np(lig.rotatable, np.uint8)
        s = Ligand()
        s.n_atoms = len(self.types)
        s.n_bonds = len(self.rot)
        s.type_id = self.types.ctypes.data_as(C.POINTER(C.c_int))
        s.charge = self.q.ctypes.data_as(C.POINTER(C.c_float))
        s.xyz = self.xyz.ctypes.data_as(C.POINTER(C.c_float))
        s.bonds = self.bonds.ctypes.data_as(C.POINTER(C.c_int)) if self.bonds.size else None
        s.rotatable = self.rot.ctypes.data_as(C.POINTER(C.c_ubyte)) if self.rot.size else None
        self.s = s


def ad_ligand_check(lig, n_types: int):
    """Host-only validation; returns (code, message)."""
    a = _LigandArrays(lig)
    buf = C.create_string_buffer(256)
    rc = lib().ad_ligand_check(C.byref(a.s), n_types, buf, 256)
    return rc, buf.value.decode()


def ad_grid_check(grid, n_types: int):
    """Host-only grid validation; returns (code, message)."""
    d, keep = _grid_desc(grid)
    buf = C.create_string_buffer(256)
    rc = lib().ad_grid_check(C.byref(d), n_types, buf, 256)
    return rc, buf.value.decode()


def _grid_desc(grid):
    mt = (C.c_int * max(1, len(grid.map_types)))(*grid.map_types)
    d = GridDesc()
    d.nx, d.ny, d.nz = grid.n
    d.spacing = grid.spacing
    d.origin[:] = list(grid.origin)
    d.n_maps = len(grid.map_types)
    d.map_types = C.cast(mt, C.POINTER(C.c_int))
    return d, mt


class Batch:
    def __init__(self, ctx, handle, n):
        self.ctx = ctx
        self.h = handle
        self.n = n
        ctx._children.add(self)

    def info(self, i):
        a, t, p, f, d = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_int()
        rc = lib().ad_batch_info(self.h, i, C.byref(a), C.byref(t), C.byref(p), C.byref(f), C.byref(d))
        if rc:
            raise AddockError(rc, "bad ligand index")
        return dict(n_atoms=a.value, n_torsions=t.value, n_pairs=p.value, n_fragments=f.value,
                    depth_sum=d.value)

    def free(self):
        if self.h:
            lib().ad_free_batch(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be gone (and
        # module globals cleared): the process is ending, the driver reclaims
        # the memory
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


_live_contexts = weakref.WeakSet()
_atexit_registered = False


def _close_all_contexts():
    """atexit: close live contexts (their batches and pre-screens first)
    while the HIP runtime is still up.  Registered after torch is imported,
    so it runs before torch's own exit handlers."""
    for ctx in list(_live_contexts):
        try:
            ctx.close()
        except Exception:
            pass


class Context:
    """One addock context (ad_create) on `device`; stream None = own stream,
    'torch' = the current torch stream."""

    def __init__(self, ff: dict, device: int = 0, stream=None):
        L = lib()
        self.ff = make_forcefield(ff)
        h = C.c_void_p()
        if stream == "torch":
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self._children = weakref.WeakSet()   # batches and pre-screens: freed before the context
        rc = L.ad_create(C.byref(h), device, C.byref(self.ff), C.c_void_p(stream) if stream else None)
        if rc:
            raise AddockError(rc, "ad_create failed")
        self.h = h
        global _atexit_registered
        _live_contexts.add(self)
        if not _atexit_registered:
            atexit.register(_close_all_contexts)
            _atexit_registered = True

    def _check(self, rc):
        if rc:
            raise AddockError(rc, lib().ad_last_error(self.h).decode())

    def ad_set_kernel_timing(self, enable: bool):
        self._check(lib().ad_set_kernel_timing(self.h, 1 if enable else 0))

    def ad_get_kernel_timing(self, reset: bool = False):
        t = KernelTimes()
        self._check(lib().ad_get_kernel_timing(self.h, C.byref(t), 1 if reset else 0))
        out = {k: (t.ms[i], int(t.launches[i])) for i, k in enumerate(KERNEL_KINDS)}
        out["busy_ms"] = {k: t.busy_ms[i] for i, k in enumerate(KERNEL_KINDS)}
        return out

    def ad_set_schedule(self, use_graph=True, autotune=True, stage_pairs=-1, pack_small=True):
        self._check(lib().ad_set_schedule(self.h, int(use_graph), int(autotune), int(stage_pairs), int(pack_small)))

    def ad_get_schedule(self):
        st = (C.c_int * 2)()
        g, pk = C.c_int(), C.c_int()
        self._check(lib().ad_get_schedule(self.h, st, C.byref(g), C.byref(pk)))
        return dict(stage_pairs=[st[0], st[1]], graph=bool(g.value), packed_runs=pk.value)

    def ad_set_launch_shape(self, unroll=0, wg_per_cu=0):
        """Force the local search's pair-loop form (1 or 2 steps per trip) and/or work-groups per CU; 0: tuned."""
        self._check(lib().ad_set_launch_shape(self.h, int(unroll), int(wg_per_cu)))

    def ad_get_launch_shape(self):
        u, w = (C.c_int * 2)(), (C.c_int * 2)()
        self._check(lib().ad_get_launch_shape(self.h, u, w))
        return dict(unroll=[u[0], u[1]], wg_per_cu=[w[0], w[1]])

    def ad_set_work_queue(self, mode=-1):
        """Persistent work queue of the generation launches: -1 tuned, 0 off, 1 on."""
        self._check(lib().ad_set_work_queue(self.h, int(mode)))

    def ad_get_work_queue(self):
        q = (C.c_int * 2)()
        self._check(lib().ad_get_work_queue(self.h, q))
        return [q[0], q[1]]

    def ad_set_chains(self, parts=2):
        """Split every bucket's runs into `parts` chains of launches on their own streams."""
        self._check(lib().ad_set_chains(self.h, int(parts)))

    MICROBENCH_KINDS = ("fma_f32_flops", "fma_f64_flops", "exp2_f32_per_s", "lds_add_f64_per_s", "gather_bytes_per_s")

    def ad_microbench(self, kind, nbytes=0):
        """Rate measured by microbenchmark `kind` (index or name of MICROBENCH_KINDS); nbytes: gather buffer."""
        k = self.MICROBENCH_KINDS.index(kind) if isinstance(kind, str) else int(kind)
        out = C.c_double()
        self._check(lib().ad_microbench(self.h, k, int(nbytes), C.byref(out)))
        return out.value

    def ad_get_chains(self):
        q = (C.c_int * 2)()
        self._check(lib().ad_get_chains(self.h, q))
        return [q[0], q[1]]

    def ad_synchronize(self):
        self._check(lib().ad_synchronize(self.h))

    def ad_set_stream(self, stream):
        self._check(lib().ad_set_stream(self.h, C.c_void_p(stream) if stream else None))

    def ad_load_grids(self, grid, maps):
        d, keep = _grid_desc(grid)
        if _is_device(maps):
            self._check(lib().ad_load_grids(self.h, C.byref(d), _ptr(maps), 1))
        else:
            m = _np(maps, np.float32)
            self._check(lib().ad_load_grids(self.h, C.byref(d), _ptr(m), 0))

    def ad_build_grids(self, grid, receptor, want_maps=False):
        d, keep = _grid_desc(grid)
        xyz = _np(receptor.xyz, np.float32).reshape(-1)
        ty = _np(receptor.types, np.int32)
        q = _np(receptor.charges, np.float32)
        out = None
        if want_maps:
            nx, ny, nz = grid.n
            out = np.empty((len(grid.map_types) + 2, nz, ny, nx), np.float32)
        self._check(lib().ad_build_grids(self.h, C.byref(d), len(ty), xyz.ctypes.data_as(C.POINTER(C.c_float)),
                                         ty.ctypes.data_as(C.POINTER(C.c_int)),
                                         q.ctypes.data_as(C.POINTER(C.c_float)),
                                         out.ctypes.data_as(C.POINTER(C.c_float)) if out is not None else None))
        return out

    def ad_load_ligands(self, ligs) -> Batch:
        if hasattr(ligs, "n_atoms_per_ligand"):   # a packed set (synth.LigandPack)
            return self.ad_load_ligands_packed(ligs)
        arrs = [_LigandArrays(l) for l in ligs]
        arr = (Ligand * max(1, len(arrs)))(*[a.s for a in arrs])
        h = C.c_void_p()
        self._check(lib().ad_load_ligands(self.h, len(arrs), arr, C.byref(h)))
        return Batch(self, h, len(arrs))

    def ad_load_ligands_packed(self, pack) -> Batch:
        na = _np(pack.n_atoms_per_ligand, np.int32)
        nb = _np(pack.n_bonds_per_ligand, np.int32)
        ty = _np(pack.types, np.int32)
        q = _np(pack.charges, np.float32)
        xyz = _np(pack.xyz, np.float32).reshape(-1)
        bd = _np(pack.bonds, np.int32).reshape(-1)
        rot = _np(pack.rotatable, np.uint8)
        h = C.c_void_p()
        self._check(lib().ad_load_ligands_packed(self.h, len(na), _ptr(na), _ptr(nb), _ptr(ty), _ptr(q), _ptr(xyz),
                                                 _ptr(bd), _ptr(rot), C.byref(h)))
        return Batch(self, h, len(na))

    def ad_score_poses(self, batch, lig_idx, genotypes, grad=False, terms=False, out=None, shape=None):
        """Host (numpy) or device (torch CUDA) arrays.  Returns (energy, grad, terms).
        shape: None (ad_score_poses) or an AD_SHAPE_* value (ad_score_poses_shape)."""
        def call(*a):
            if shape is None:
                return lib().ad_score_poses(*a)
            return lib().ad_score_poses_shape(*a, int(shape))
        if _is_device(genotypes):
            import torch
            n = genotypes.shape[0]
            E = out["energy"] if out else torch.empty(n, dtype=torch.float32, device=genotypes.device)
            G = (out["grad"] if out else torch.empty((n, STRIDE), dtype=torch.float32,
                                                     device=genotypes.device)) if grad else None
            T = (out["terms"] if out else torch.empty((n, 3), dtype=torch.float32,
                                                      device=genotypes.device)) if terms else None
            self._check(call(self.h, batch.h, n, _ptr(lig_idx), _ptr(genotypes), _ptr(E), _ptr(G), _ptr(T), 1))
            return E, G, T
        g = _np(genotypes, np.float32)
        n = g.shape[0]
        idx = _np(lig_idx, np.int32)
        E = np.empty(n, np.float32)
        G = np.empty((n, STRIDE), np.float32) if grad else None
        T = np.empty((n, 3), np.float32) if terms else None
        self._check(call(self.h, batch.h, n, _ptr(idx), _ptr(g), _ptr(E), _ptr(G), _ptr(T), 0))
        return E, G, T

    def ad_score_poses_noalloc(self, batch, lig_idx, genotypes, grad=False, terms=False):
        """Host (numpy) arrays only, at most NOALLOC_MAX_POSES poses: ad_score_poses staged through
        the library's static device block.  Returns (energy, grad, terms)."""
        g = _np(genotypes, np.float32)
        n = g.shape[0]
        idx = _np(lig_idx, np.int32)
        E = np.empty(n, np.float32)
        G = np.empty((n, STRIDE), np.float32) if grad else None
        T = np.empty((n, 3), np.float32) if terms else None
        self._check(lib().ad_score_poses_noalloc(self.h, batch.h, n, _ptr(idx), _ptr(g), _ptr(E), _ptr(G), _ptr(T)))
        return E, G, T

    def ad_local_search(self, batch, lig_idx, genotypes, params: DockParams, iters: int, shape=None):
        """Host arrays: returns (best genotypes, energies); device tensors are updated in place.
        shape: None (ad_local_search) or an AD_SHAPE_* value (ad_local_search_shape)."""
        def call(*a):
            if shape is None:
                return lib().ad_local_search(*a)
            return lib().ad_local_search_shape(*a, int(shape))
        if _is_device(genotypes):
            import torch
            n = genotypes.shape[0]
            E = torch.empty(n, dtype=torch.float32, device=genotypes.device)
            self._check(call(self.h, batch.h, n, _ptr(lig_idx), _ptr(genotypes), _ptr(E), C.byref(params), iters, 1))
            return genotypes, E
        g = _np(genotypes, np.float32).copy()
        n = g.shape[0]
        idx = _np(lig_idx, np.int32)
        E = np.empty(n, np.float32)
        self._check(call(self.h, batch.h, n, _ptr(idx), _ptr(g), _ptr(E), C.byref(params), iters, 0))
        return g, E

    def ad_solis_wets(self, batch, lig_idx, genotypes, params: DockParams, max_evals: int, seed: int):
        """Host arrays: returns (best genotypes, energies, evaluations used)."""
        g = _np(genotypes, np.float32).copy()
        n = g.shape[0]
        idx = _np(lig_idx, np.int32)
        E = np.empty(n, np.float32)
        used = np.empty(n, np.int32)
        self._check(lib().ad_solis_wets(self.h, batch.h, n, _ptr(idx), _ptr(g), _ptr(E), _ptr(used), C.byref(params),
                                        max_evals, seed))
        return g, E, used

    def ad_dock_batch(self, batch, params: DockParams, seed: int, lig_ids=None, per_run=False):
        n = batch.n
        res = (DockResult * max(1, n))()
        ids = _np(lig_ids, np.uint32) if lig_ids is not None else None
        re = np.empty((n, params.nrun), np.float32) if per_run else None
        rg = np.empty((n, params.nrun, STRIDE), np.float32) if per_run else None
        self._check(lib().ad_dock_batch(self.h, batch.h, C.byref(params), seed, _ptr(ids), res,
                                        re.ctypes.data_as(C.POINTER(C.c_float)) if per_run else None,
                                        rg.ctypes.data_as(C.POINTER(C.c_float)) if per_run else None))
        return self._results(res, n, re, rg, per_run)

    def ad_dock_select(self, batch, lig_idx, params: DockParams, seed: int, per_run=False):
        idx = _np(lig_idx, np.int32)
        n = len(idx)
        res = (DockResult * max(1, n))()
        re = np.empty((n, params.nrun), np.float32) if per_run else None
        rg = np.empty((n, params.nrun, STRIDE), np.float32) if per_run else None
        self._check(lib().ad_dock_select(self.h, batch.h, n, _ptr(idx), C.byref(params), seed, res,
                                         re.ctypes.data_as(C.POINTER(C.c_float)) if per_run else None,
                                         rg.ctypes.data_as(C.POINTER(C.c_float)) if per_run else None))
        return self._results(res, n, re, rg, per_run)

    def ad_dock_stream(self, pack, batch_size: int, params: DockParams, seed: int, id0: int = 0):
        """Dock a back-to-back ligand set (synth.LigandPack layout) in batches
        of batch_size, host preparation of the next batch overlapping the
        docking of the current one; ligand i uses random-stream id id0 + i."""
        na = _np(pack.n_atoms_per_ligand, np.int32)
        nb = _np(pack.n_bonds_per_ligand, np.int32)
        ty = _np(pack.types, np.int32)
        q = _np(pack.charges, np.float32)
        xyz = _np(pack.xyz, np.float32).reshape(-1)
        bd = _np(pack.bonds, np.int32).reshape(-1)
        rot = _np(pack.rotatable, np.uint8)
        n = len(na)
        res = (DockResult * max(1, n))()
        st = (C.c_double * 3)()
        self._check(lib().ad_dock_stream(self.h, n, _ptr(na), _ptr(nb), _ptr(ty), _ptr(q), _ptr(xyz), _ptr(bd),
                                         _ptr(rot), int(batch_size), C.byref(params), seed, int(id0), res, st))
        out = self._results(res, n, None, None, False)
        out["stats"] = dict(prep_s=st[0], dock_s=st[1], wall_s=st[2])
        return out

    @staticmethod
    def _results(res, n, re, rg, per_run):
        dt = np.dtype({"names": ["best_energy", "best_score", "best_genotype", "best_run", "generations", "evals"],
                       "formats": ["<f4", "<f4", ("<f4", (STRIDE,)), "<i4", "<i4", "<i8"],
                       "offsets": [DockResult.best_energy.offset, DockResult.best_score.offset,
                                   DockResult.best_genotype.offset, DockResult.best_run.offset,
                                   DockResult.generations.offset, DockResult.evals.offset],
                       "itemsize": C.sizeof(DockResult)})
        a = np.frombuffer(res, dtype=dt, count=n)
        out = dict(best_energy=a["best_energy"].copy(), best_score=a["best_score"].copy(),
                   best_genotype=a["best_genotype"].copy(), best_run=a["best_run"].copy(),
                   generations=a["generations"].copy(), evals=a["evals"].copy())
        if per_run:
            out["run_energy"] = re
            out["run_genotype"] = rg
        return out

    def ad_initial_population(self, batch, lig, lig_id, run, pop, seed):
        g = np.empty((pop, STRIDE), np.float32)
        self._check(lib().ad_initial_population(self.h, batch.h, lig, lig_id, run, pop, seed,
                                                g.ctypes.data_as(C.POINTER(C.c_float))))
        return g

    def close(self):
        """Free the batches and pre-screens still open, then the context.  The
        library detaches any child it still finds, so the order is not needed
        for safety; it only releases their memory early."""
        if getattr(self, "h", None):
            for child in list(self._children):
                child.close() if isinstance(child, Prescreen) else child.free()
            lib().ad_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


class Prescreen:
    """The learned pre-screen (ad_prescreen_*) on a context's device."""

    def __init__(self, ctx: Context, seed: int = 0, **cfg):
        d = dict(DEFAULT_PRESCREEN)
        d.update(cfg)
        c = PrescreenCfg()
        for k, v in d.items():
            setattr(c, k, v)
        self.ctx = ctx
        h = C.c_void_p()
        ctx._check(lib().ad_prescreen_create(ctx.h, C.byref(c), seed, C.byref(h)))
        self.h = h
        ctx._children.add(self)
        self.n_params = lib().ad_prescreen_n_params()

    def ad_prescreen_set_params(self, params):
        p = _np(params, np.float32)
        assert p.size == self.n_params
        self.ctx._check(lib().ad_prescreen_set_params(self.h, _fptr(p)))

    def ad_prescreen_get_params(self):
        p = np.empty(self.n_params, np.float32)
        self.ctx._check(lib().ad_prescreen_get_params(self.h, _fptr(p)))
        return p

    def ad_prescreen_set_scale(self, mean, sd):
        self.ctx._check(lib().ad_prescreen_set_scale(self.h, float(mean), float(sd)))

    def ad_prescreen_get_scale(self):
        m, s = C.c_double(), C.c_double()
        self.ctx._check(lib().ad_prescreen_get_scale(self.h, C.byref(m), C.byref(s)))
        return m.value, s.value

    def ad_prescreen_predict(self, batch, lig_idx=None):
        idx = _np(lig_idx, np.int32) if lig_idx is not None else None
        n = len(idx) if idx is not None else batch.n
        out = np.empty(n, np.float32)
        self.ctx._check(lib().ad_prescreen_predict(self.h, batch.h, n, _ptr(idx), _fptr(out)))
        return out

    def ad_prescreen_grad(self, batch, lig_idx, labels):
        idx = _np(lig_idx, np.int32)
        y = _np(labels, np.float32)
        n = len(idx)
        loss = np.zeros(1, np.float32)
        grad = np.empty(self.n_params, np.float32)
        pred = np.empty(n, np.float32)
        self.ctx._check(lib().ad_prescreen_grad(self.h, batch.h, n, _ptr(idx), _fptr(y), _fptr(loss), _fptr(grad),
                                                _fptr(pred)))
        return float(loss[0]), grad, pred

    def ad_prescreen_train(self, batch, lig_idx, labels, epochs, seed=0):
        idx = _np(lig_idx, np.int32) if lig_idx is not None else None
        y = _np(labels, np.float32)
        n = len(y)
        curve = np.zeros(max(1, epochs), np.float32)
        self.ctx._check(lib().ad_prescreen_train(self.h, batch.h, n, _ptr(idx), _fptr(y), epochs, seed,
                                                 _fptr(curve)))
        return curve[:epochs]

    def close(self):
        if getattr(self, "h", None):
            lib().ad_prescreen_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def create(ff: dict, device: int = 0, stream=None) -> Context:
    return Context(ff, device, stream)
