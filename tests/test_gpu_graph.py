"""Graph launches (mpcd_set_graph): the kernels of each stepping call
captured into a HIP graph and launched as one. The state after any sequence
of calls equals the same calls launched kernel by kernel on the stream, bit
for bit: one box in both forms and both collision rules, a batch, the
enlarge-and-replay path after a slab overflow, and calls made while kernel
timing is on (those launch on the stream). The context keeps its executable
graph: a call of the same shape as the last updates it in place."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import banner

pytestmark = pytest.mark.gpu

CALLS = [5, 7, 7, 7, 3, 1, 1, 4]


def _run(make, graph, calls=CALLS, profile=False):
    with make() as s:
        s.set_graph(graph)
        if profile:
            s.profile(True, every=2)
        for n in calls:
            s.step(n)
        pos, vel = s.get_state()
        cells, counts = s.get_cells()
        stats = s.graph_stats()
        layout = s.layout()
    return pos, vel, cells, counts, stats, layout


def _same(a, b):
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec,rule", [(m.FP32, m.SRD), (m.FP64, m.SRD), (m.FP32, m.AT),
                                       (m.FP64, m.AT)])
def test_graph_equals_stream_one_box(prec, rule):
    banner(f"graph vs stream, one box, prec {prec} rule {rule}")
    pos, vel = workloads.fluid((12, 10, 9), 9.0, seed=31)

    def make():
        return m.Sim(pos, vel, (12, 10, 9), seed=32, precision=prec,
                     thermostat=rule == m.SRD, collision=rule)
    a = _run(make, False)
    b = _run(make, True)
    _same(a, b)
    inst, upd = b[4]
    assert a[4] == (0, 0)
    # shapes: 5 steps from create (with the first stream + bin), 7, 3, 1, 4
    # steps adopting a prepared binning; the repeats update in place
    assert inst + upd == len(CALLS) and upd >= 3
    print(f"graph instantiations {inst}, in-place updates {upd}")


def test_graph_equals_stream_batch():
    banner("graph vs stream, batch")
    boxes = workloads.replica_inputs(workloads.replica_boxes(6, seed=3, side=(5, 14)))

    def make():
        return m.Batch(boxes, precision=m.FP32, thermostat=True)
    _same(_run(make, False), _run(make, True))


def test_graph_equals_stream_slab_regrow():
    """A converging flow overflows tight slabs inside graph-launched calls:
    the replay from the failing launch gives the stream's result."""
    banner("graph vs stream, slab regrow")
    pos, vel = workloads.fluid((12, 12, 12), 9, seed=96)
    vel = vel - (pos - 6.0)

    def make():
        return m.Sim(pos, vel, (12, 12, 12), seed=95, precision=m.FP32, thermostat=True,
                     flags=m.binding.FLAG_TIGHT_SLABS)
    a = _run(make, False, calls=[2, 2, 2])
    b = _run(make, True, calls=[2, 2, 2])
    assert a[5][3] >= 1 and b[5][3] == a[5][3]
    _same(a, b)


def test_graph_with_kernel_timing_launches_on_the_stream():
    banner("graph with kernel timing")
    pos, vel = workloads.fluid((8, 8, 8), 10.0, seed=41)

    def make():
        return m.Sim(pos, vel, (8, 8, 8), seed=42, precision=m.FP32, thermostat=True)
    a = _run(make, False)
    b = _run(make, True, profile=True)
    _same(a, b)
    assert b[4] == (0, 0)


def test_graph_switch_takes_0_or_1():
    pos, vel = workloads.fluid((4, 4, 4), 5.0, seed=1)
    with m.Sim(pos, vel, (4, 4, 4)) as s:
        with pytest.raises(m.MpcdError):
            m.binding._check(m.binding.load().mpcd_set_graph(s._ctx, 2))
