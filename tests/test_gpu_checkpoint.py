"""Checkpoints through the C ABI (iblb_state_size / iblb_save_state /
iblb_load_state): a run resumed from a saved state continues bit for bit
like the run that saved it, in a fresh context or in the same one rewound,
with every storage and with the viscosity contrast and moving walls."""
import numpy as np
import pytest

from iblb_inputs import configs

from _helpers import say

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = 0, 1, 2, 3
GRAPH = 1


def sim(wl, storage, flags=GRAPH):
    import paper_2604_17463_amd as P
    return P.Simulation(wl, storage=storage, flags=flags,
                        dev_scale=4096.0 if storage == F16 else 1.0)


def _snapshot(s):
    drops, boxes = s.observables()
    return s.read_state(0), s.read_nodes(0), drops[0], boxes[0]


def _same(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    for k in ("step", "volume", "area", "height", "contact_radius", "deformation"):
        assert a[2][k] == b[2][k], k
    assert a[3]["mass"] == b[3]["mass"]


def _workloads():
    yield "c1", configs.plain_c1()
    c1c = configs.plain_c1()
    c1c.boxes[0].tau_in = 1.4
    yield "c1-contrast", c1c
    yield "shear", configs.shear_droplet(lam=2.0, r=6.0, ca=0.2, re=0.5, shape=(32, 24, 32), level=3)


@pytest.mark.parametrize("storage", [F64, F32, F16, BF16])
@pytest.mark.parametrize("name", ["c1", "c1-contrast", "shear"])
def test_resume_in_a_fresh_context_is_bitwise(name, storage):
    say("checkpoint fresh context", name, storage)
    wl = dict(_workloads())[name]
    a = sim(wl, storage)
    a.step(50)
    blob = a.save_state()
    a.step(31)
    want = _snapshot(a)
    b = sim(wl, storage)
    b.step(3)                     # a context that has run does not matter
    b.load_state(blob)
    b.step(31)
    _same(_snapshot(b), want)
    assert want[2]["step"] == 81


def test_rewinding_the_same_context_is_bitwise():
    say("checkpoint rewind")
    wl = configs.plain_c1()
    s = sim(wl, F32)
    s.step(40)
    blob = s.save_state()
    s.step(37)
    first = _snapshot(s)
    s.load_state(blob)            # 37 steps later: the other buffer parity
    s.step(37)
    _same(_snapshot(s), first)


def test_load_rejects_another_configuration():
    import paper_2604_17463_amd as P
    say("checkpoint mismatch")
    a = sim(configs.plain_c1(), F32)
    blob = a.save_state()
    other = configs.plain_c1()
    other.boxes[0].tau = 0.9
    b = sim(other, F32)
    with pytest.raises(P.IblbError):
        b.load_state(blob)
    c = sim(configs.plain_c1(), F64)
    with pytest.raises(P.IblbError):
        c.load_state(blob)
    with pytest.raises(P.IblbError):
        a.load_state(blob[:-8])
    bad = bytearray(blob)
    bad[0] ^= 1
    with pytest.raises(P.IblbError):
        a.load_state(bytes(bad))
