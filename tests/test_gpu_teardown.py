"""Teardown on the GPU: contexts, batches and pre-screens released in any
order.  ad_destroy detaches the children still alive, so a batch or
pre-screen freed after its context only deletes the handle.  The scenarios run
in a child process (a crash at exit would otherwise be invisible to the test
that caused it): children freed after their context through the raw C ABI,
reference cycles collected by the garbage collector, and live cycles left for
interpreter exit.  The process must exit with status 0."""
import os
import subprocess
import sys
import textwrap

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import ctypes as C, gc, sys
    sys.path.insert(0, {root!r})
    import numpy as np
    import torch
    import paper_2007_03678_amd as pkg
    import synth
    ff = synth.forcefield()
    grid = synth.make_grid(16, 0.5, map_types=synth.SIX_TYPES)
    maps = np.zeros((len(grid.map_types) + 2, 16, 16, 16), np.float32)
    ligs = [synth.ligand(1, 20, 4), synth.ligand(2, 30, 6)]

    def make():
        ctx = pkg.create(ff, 0)
        ctx.ad_load_grids(grid, maps)
        batch = ctx.ad_load_ligands(ligs)
        ps = pkg.Prescreen(ctx, seed=1)
        return ctx, batch, ps

    # 1. children freed after the context, through the C ABI
    ctx, batch, ps = make()
    L = pkg.lib()
    L.ad_destroy(ctx.h); ctx.h = None
    g = np.zeros((1, 40), np.float32); g[0, 3] = 1
    E = np.zeros(1, np.float32); idx = np.zeros(1, np.int32)
    ctx2 = pkg.create(ff, 0)   # a live context does not accept the detached batch
    ctx2.ad_load_grids(grid, maps)
    rc = L.ad_score_poses(ctx2.h, batch.h, 1, idx.ctypes.data, g.ctypes.data, E.ctypes.data, None, None, 0)
    assert rc == pkg.AD_E_INVALID, rc
    ctx2.close()
    out = np.zeros(2, np.float32)
    assert L.ad_prescreen_predict(ps.h, batch.h, 2, None, out.ctypes.data_as(C.POINTER(C.c_float))) == pkg.AD_E_INVALID
    batch.free(); ps.close()
    print("detached ok", flush=True)
    # 2. reference cycles collected in the collector's order
    for k in range(5):
        ctx, batch, ps = make()
        ctx.cycle = [batch, ps]; batch.cycle = ps.cycle = ctx
        del ctx, batch, ps
        gc.collect()
    torch.cuda.synchronize()
    print("cycles ok", flush=True)
    # 3. live cycles left for interpreter exit
    ctx, batch, ps = make()
    ctx.cycle = [batch, ps]; batch.cycle = ctx
    keep = make()
    print("exit", flush=True)
""")


def test_teardown_in_any_order_exits_cleanly():
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT)], capture_output=True, text=True,
                       timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    assert "Exception ignored" not in r.stderr, r.stderr[-2000:]
    for tag in ("detached ok", "cycles ok", "exit"):
        assert tag in r.stdout
