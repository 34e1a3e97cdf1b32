"""The microbenchmarks behind the roofline peaks (ad_microbench): every kind
returns a finite positive rate, and the vector FMA rates come out within
reach of the published figures (FP32 157.3 TFLOP/s, FP64 78.6 TFLOP/s) and
below them."""
import math

import pytest

pytestmark = pytest.mark.gpu


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


def test_rates_are_finite_and_fma_near_the_published_rate(ctx):
    r = {k: ctx.ad_microbench(k, 1 << 22 if k.startswith("gather") else 0) for k in ctx.MICROBENCH_KINDS}
    for k, v in r.items():
        assert math.isfinite(v) and v > 0, (k, v)
    assert 0.4 * 157.3e12 < r["fma_f32_flops"] < 1.05 * 157.3e12, r
    assert 0.4 * 78.6e12 < r["fma_f64_flops"] < 1.05 * 78.6e12, r
    # a transcendental issues at a quarter of the FMA rate or faster
    assert r["exp2_f32_per_s"] > 0.2 * r["fma_f32_flops"] / 2 / 4
    big = ctx.ad_microbench("gather_bytes_per_s", 32 << 20)
    assert math.isfinite(big) and big > 0


def test_bad_arguments_are_rejected(pkg, ctx):
    with pytest.raises(pkg.AddockError):
        ctx.ad_microbench(5)
    with pytest.raises(pkg.AddockError):
        ctx.ad_microbench("gather_bytes_per_s", 100)
