"""The entry point that allocates nothing, sbt_create_static, against
sbt_create on the same cases: the same kernels on memory from the library's
static device array instead of a caller buffer must give the same bits.  Two
contexts in a row (the second smaller) reuse the array; too large a case
and a second live context on the device are rejected."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2402_04606_amd as pkg
    pkg.lib()
    return pkg


def _run(P, wl, steps, static):
    print(f"case {wl.name} steps {steps} static {static}", flush=True)
    g = P.Sim(wl, "f64", static_memory=static)
    g.step(steps)
    g.synchronize()
    out = [g.fields_blocks(0, l) for l in range(wl.n_levels)]
    hist = g.force_history() if wl.body is not None else None
    g.close()
    return out, hist


def test_static_context_matches_allocated_one_twice(P):
    for wl, steps in ((W.small_refined_flap(), 6), (W.tgv(32, tau=0.7), 40)):
        a, ha = _run(P, wl, steps, False)
        b, hb = _run(P, wl, steps, True)
        for x, y in zip(a, b):
            assert np.array_equal(x, y, equal_nan=True)
        if ha is not None:
            assert np.array_equal(ha[0], hb[0]) and np.array_equal(ha[1], hb[1])


def test_static_context_limits(P):
    with pytest.raises(P.SbtError) as e:
        P.Sim(W.batch_sweep(), "f16s", static_memory=True)      # 772 MiB > 128 MiB
    assert e.value.code == -4
    g = P.Sim(W.tgv(32), "f64", static_memory=True)
    with pytest.raises(P.SbtError) as e:
        P.Sim(W.tgv(32), "f64", static_memory=True)              # the array is in use
    assert e.value.code == -5
    g.close()
    h = P.Sim(W.tgv(32), "f64", static_memory=True)              # free again after sbt_destroy
    h.step(2)
    h.synchronize()
    h.close()
