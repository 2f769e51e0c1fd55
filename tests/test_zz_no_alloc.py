"""The observables entry point that allocates nothing (lb_observables_static,
for callers that cannot allocate device memory) against lb_observables: the
same kernels and summation order, so the same bits, on two calls in a row,
the second on a smaller input; and a clear error when the boxes need more
partial sums than its static array holds."""
from __future__ import annotations

import numpy as np
import pytest

from lbtest import chain, gpu_system, params, say

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0903_5067_amd as lbm
    lbm.lib()


def _same(a, b):
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k
        else:
            assert a[k] == b[k], k


def test_static_observables_equal_the_allocating_ones_on_two_calls():
    import paper_0903_5067_amd as lbm
    say("static observables: larger input")
    big = [params(L=24, N=16, kT=1e-2, box_id=0), params(L=40, N=300, kT=1e-2, box_id=1),
           params(L=16, N=0, kT=1e-2, box_id=2)]
    s1 = gpu_system(big, FP32, xs=[chain(b) for b in big])
    s1.set_launch(batched=True, graph_steps=0)
    s1.step(12)
    o_static = s1.observables(static=True)
    o_ref = s1.observables()
    for a, b in zip(o_static, o_ref):
        _same(a, b)
    assert o_ref[1]["rg2"] > 0 and o_ref[2]["mass"] > 0
    s1.close()
    say("static observables: smaller input, FP64")
    small = [params(L=8, N=4, kT=1e-3, box_id=5)]
    s2 = gpu_system(small, FP64, xs=[chain(b) for b in small])
    s2.step(5)
    o_static = s2.observables(static=True)
    o_ref = s2.observables()
    _same(o_static[0], o_ref[0])
    s2.close()


def test_static_observables_reject_too_many_partials():
    import paper_0903_5067_amd as lbm
    say("static observables: too many boxes")
    boxes = [params(L=2, N=0, box_id=i) for i in range(700)]
    s = gpu_system(boxes, FP32)
    with pytest.raises(lbm.LBError) as e:
        s.observables(static=True)
    assert e.value.status == lbm.LB_ENOMEM and "static array" in str(e.value)
    assert len(s.observables()) == 700   # the allocating entry point still serves them
    s.close()
