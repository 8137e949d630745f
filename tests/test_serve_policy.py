"""Host logic of the server's per-request precision policy (no GPU)."""
import fde_inputs as fi
from paper_1912_13304_amd import fde, serve


def test_auto_precision_by_request_class():
    p1 = fi.variable_1d(n=1023, steps=2)
    p2 = fi.variable_2d(n=511, steps=2)
    p3 = fi.variable_2d(n=255, steps=2)
    kw = dict(precision=serve.AUTO, inner_steps=16, restart=30)
    k1 = serve.request_kw(p1, kw)
    k2 = serve.request_kw(p2, kw)
    k3 = serve.request_kw(p3, kw)
    assert k1["precision"] == fde.FP64 and "inner_steps" not in k1 and k1["restart"] == 30
    assert k2["precision"] == fde.MIXED and k2["inner_steps"] == 16
    assert k3["precision"] == fde.FP64 and "inner_steps" not in k3   # small 2D grids: float64
    assert kw["precision"] == serve.AUTO   # the caller's options are not modified
    # an explicit precision is kept for every request
    for p in (p1, p2, p3):
        assert serve.request_kw(p, dict(precision=fde.MIXED))["precision"] == fde.MIXED
        fde.params_for(p, **serve.request_kw(p, kw))   # valid parameter sets


def test_auto_inner_steps_by_request_class():
    p1 = fi.variable_1d(n=1023, steps=2)
    p2 = fi.variable_2d(n=63, steps=2)
    kw = dict(precision=fde.MIXED, inner_steps=serve.AUTO)
    assert serve.request_kw(p1, kw) == dict(precision=fde.MIXED, inner_steps=0)
    assert serve.request_kw(p2, kw) == dict(precision=fde.MIXED, inner_steps=serve.INNER_2D)
    # float64 requests take no inner length
    assert serve.request_kw(p1, dict(precision=serve.AUTO, inner_steps=serve.AUTO)) == dict(precision=fde.FP64)
    for p in (p1, p2):
        fde.params_for(p, **serve.request_kw(p, kw))
