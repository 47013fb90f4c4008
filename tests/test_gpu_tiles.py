"""Tile shapes set through the flags (MPCD_TILE_*) instead of the density
rule: results do not depend on the shape, bit for bit (exact cell sums,
per-particle random numbers keyed on cell and tag), in one box and in a
batch whose boxes take different shapes; the tuner times the shapes and
caches its choice."""
import json

import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import banner
from paper_1801_10187_amd import autotune

pytestmark = pytest.mark.gpu

SHAPES = list(m.binding.TILE_SHAPES)
DIMS = {"4x4x2": (4, 4, 2), "4x4x4": (4, 4, 4), "8x4x4": (8, 4, 4), "8x8x4": (8, 8, 4)}


@pytest.mark.parametrize("prec,rule", [(m.FP32, m.SRD), (m.FP64, m.SRD), (m.FP32, m.AT),
                                       (m.FP64, m.AT)])
def test_every_shape_gives_the_same_steps(prec, rule):
    banner(f"tile shapes, prec {prec} rule {rule}")
    n_cells = (20, 18, 13)
    pos, vel = workloads.fluid(n_cells, 6.0, seed=51)
    out = {}
    for shape in [None] + SHAPES:
        with m.Sim(pos, vel, n_cells, seed=52, precision=prec, thermostat=rule == m.SRD,
                   collision=rule, tile=shape) as s:
            tile = s.layout()[0]
            assert shape is None or tuple(tile) == DIMS[shape]
            s.step(3)
            s.step(2)
            out[shape] = s.get_state() + s.get_cells()
    for shape in SHAPES:
        for x, y in zip(out[None], out[shape]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("prec,rule", [(m.FP32, m.SRD), (m.FP64, m.SRD), (m.FP32, m.AT),
                                       (m.FP64, m.AT)])
def test_density_rule_matches_the_tuner_table(prec, rule):
    """The library's own choice of shape for a box alone (flags 0) is the one
    autotune.rule_shape names for the density, rule and form."""
    banner(f"density rule, prec {prec} rule {rule}")
    n_cells = (20, 18, 13)
    for rho in (1.5, 3.0, 5.0, 9.0, 13.0):
        pos, vel = workloads.fluid(n_cells, rho, seed=int(10 * rho))
        with m.Sim(pos, vel, n_cells, precision=prec, thermostat=rule == m.SRD,
                   collision=rule) as s:
            tile = tuple(s.layout()[0])
        want = autotune.rule_shape(pos.shape[0] / np.prod(n_cells), True, rule, prec)
        assert tile == DIMS[want], (rho, tile, want)


def test_batch_boxes_with_their_own_shapes():
    banner("tile shapes per box in a batch")
    boxes = workloads.replica_inputs(workloads.replica_boxes(4, seed=5, side=(6, 16)))
    with m.Batch(boxes, precision=m.FP32, thermostat=True) as b:
        b.step(4)
        ref = b.get_state() + b.get_cells()
    mixed = [dict(bx, tile=SHAPES[i % len(SHAPES)]) for i, bx in enumerate(boxes)]
    with m.Batch(mixed, precision=m.FP32, thermostat=True) as b:
        b.step(4)
        got = b.get_state() + b.get_cells()
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)


def test_tuner_times_every_shape_and_caches(tmp_path):
    banner("tile tuner")
    cache = str(tmp_path / "tiles.json")
    best = autotune.tune(6.0, cache=cache, n_cells=(24, 24, 24), steps=10, warmup=2, repeats=1)
    assert best in SHAPES
    rec = json.load(open(cache))
    (entry,) = rec.values()
    assert entry["best"] == best and set(entry["ms_per_step"]) == set(SHAPES)
    # a second call answers from the cache
    assert autotune.tune(6.0, cache=cache, n_cells=(24, 24, 24), steps=10) == best
