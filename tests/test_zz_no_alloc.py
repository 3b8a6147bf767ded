"""iblb_step_static (the step variant for callers that cannot allocate, with
its step scratch in the library's fixed device array) against iblb_step,
through the C ABI: bit for bit, on two calls in a row, the second on a
smaller configuration (the fixed array then holds the first call's
contents), and interleaved with iblb_step on one context.  A configuration
beyond the fixed array is refused."""
import numpy as np
import pytest

from iblb_inputs import configs

from _helpers import say

pytestmark = pytest.mark.gpu

F64, F32, GRAPH, FULL_U = 0, 1, 1, 4


def _same(a, b):
    fa, ua = a.read_state(0, want_u=True)
    fb, ub = b.read_state(0, want_u=True)
    assert np.array_equal(fa, fb)
    assert np.array_equal(ua, ub, equal_nan=True)
    for d in range(len(a.wl.droplets)):
        assert np.array_equal(a.read_nodes(d), b.read_nodes(d)), d
    oa, ba = a.observables()
    ob, bb = b.observables()
    assert [o["height"] for o in oa] == [o["height"] for o in ob]
    assert ba[0]["mass"] == bb[0]["mass"] and ba[0]["status_bits"] == bb[0]["status_bits"] == 0


@pytest.mark.parametrize("storage", [F32, F64])
def test_step_static_equals_step_on_two_calls_the_second_smaller(storage):
    import paper_2604_17463_amd as P
    for wl, n in ((configs.spreading_c2(steps=40), 40), (configs.plain_c1(), 25)):
        say("step_static vs step", wl.name, storage, n)
        ref = P.Simulation(wl, storage=storage, flags=GRAPH)
        got = P.Simulation(wl, storage=storage, flags=GRAPH)
        ref.step(n)
        got.step_static(n)
        _same(ref, got)
        ref.close()
        got.close()


def test_step_static_interleaves_with_step():
    import paper_2604_17463_amd as P
    say("step_static interleaved with step")
    wl = configs.plain_c1()
    ref = P.Simulation(wl, storage=F32, flags=GRAPH)
    got = P.Simulation(wl, storage=F32, flags=GRAPH)
    ref.step(30)
    got.step(7)
    got.step_static(9)
    got.step(11)
    got.step_static(3)
    _same(ref, got)


def test_step_static_refuses_a_configuration_beyond_the_fixed_scratch():
    import paper_2604_17463_amd as P
    say("step_static size limit")
    wl = configs.paper_spreading(0.732)
    s = P.Simulation(wl, storage=F32, flags=GRAPH)
    with pytest.raises(P.IblbError) as e:
        s.step_static(1)
    assert e.value.code == P.IBLB_E_WORKSPACE
    s.step(2)  # the context is unaffected
