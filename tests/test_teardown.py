"""Teardown of the Python binding against a stub of the library's ownership
calls (no GPU).  The stub keeps the header's contract -- a context detaches
its live batches and pre-screens when destroyed -- and aborts on any call with
a handle that was already freed.  Objects are left in reference cycles (as a
failed test's traceback holds them), collected by the garbage collector and
dropped at interpreter exit; every path must end with no live handle and no
abort."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STUB_SRC = os.path.join(ROOT, "tests", "stub", "teardown_stub.c")

SETUP = textwrap.dedent("""
    import ctypes as C, gc, sys
    sys.path.insert(0, {root!r})
    import paper_2007_03678_amd as pkg
    L = C.CDLL({lib!r})
    vp = C.c_void_p
    L.ad_create.argtypes = [C.POINTER(vp), C.c_int, vp, vp]
    L.ad_destroy.argtypes = [vp]; L.ad_destroy.restype = None
    L.ad_last_error.argtypes = [vp]; L.ad_last_error.restype = C.c_char_p
    L.stub_new_batch.argtypes = [vp, C.POINTER(vp)]
    L.ad_free_batch.argtypes = [vp]; L.ad_free_batch.restype = None
    L.ad_prescreen_create.argtypes = [vp, vp, C.c_uint64, C.POINTER(vp)]
    L.ad_prescreen_destroy.argtypes = [vp]; L.ad_prescreen_destroy.restype = None
    pkg._lib = L
    import synth
    ff = synth.forcefield()

    def make():
        ctx = pkg.Context(ff)
        h = vp()
        L.stub_new_batch(ctx.h, C.byref(h))
        batch = pkg.Batch(ctx, h, 1)
        ps = pkg.Prescreen(ctx)
        return ctx, batch, ps
""")


@pytest.fixture(scope="module")
def stub(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("stub") / "libstub.so")
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", STUB_SRC, "-o", out], check=True)
    return out


def run(stub, body):
    code = SETUP.format(root=ROOT, lib=stub) + textwrap.dedent(body)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)


def test_cycle_collected_in_any_order(stub):
    r = run(stub, """
        for k in range(20):
            ctx, batch, ps = make()
            ctx.cycle = [batch, ps, ctx]      # a reference cycle through all three
            batch.cycle = ps.cycle = ctx
            del ctx, batch, ps
            gc.collect()
        assert L.stub_live() == 0, L.stub_live()
        print("ok")
    """)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr


def test_children_freed_after_context(stub):
    r = run(stub, """
        ctx, batch, ps = make()
        L.ad_destroy(ctx.h)            # the context goes first (as a collector may order it)
        ctx.h = None
        batch.free(); ps.close()       # detached handles are only deleted
        batch.free(); ps.close()       # and a second free is a no-op in the binding
        assert L.stub_live() == 0
        print("ok")
    """)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr


def test_exit_with_live_cycle(stub):
    # objects still alive at interpreter exit: the atexit hook closes them
    # (children first); finalisers that run later make no library call
    r = run(stub, """
        import atexit
        atexit.register(lambda: print("live", L.stub_live()))   # runs after the binding's hook
        ctx, batch, ps = make()
        ctx.cycle = [batch, ps]
        batch.cycle = ctx
        ctx2, batch2, ps2 = make()
    """)
    assert r.returncode == 0, r.stderr
    assert "live 0" in r.stdout, r.stdout
    assert "Exception ignored" not in r.stderr, r.stderr
