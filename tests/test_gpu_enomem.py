"""Device memory running out (MPCD_ENOMEM), forced from the host with the
library's allocation-failure hook: every allocation of mpcd_create failing
in turn leaves nothing allocated and the next create works; a slab that
overflows when the slabs cannot be enlarged rolls the context back to the
failing launch's input, from which the run continues to the result of a
run that never failed, bit for bit; readbacks whose staging cannot be
allocated fail cleanly."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import PoolHighWater, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _hook_off():
    yield
    m.binding.debug_fail_allocs(-1)


@pytest.mark.parametrize("prec", [m.FP32, m.FP64])
def test_every_create_allocation_failing(prec):
    banner(f"create with failing allocations, prec {prec}")
    pos, vel = workloads.fluid((9, 8, 7), 6.0, seed=61)
    bpos, bvel, bmass = workloads.beads((9, 8, 7), 2, 5, seed=62)
    hw = PoolHighWater()
    kw = dict(seed=63, precision=prec, thermostat=True, emb_pos=bpos, emb_vel=bvel,
              emb_mass=bmass)
    failed = 0
    for k in range(40):
        m.binding.debug_fail_allocs(k, 1)
        try:
            s = m.Sim(pos, vel, (9, 8, 7), **kw)
        except m.MpcdError as e:
            assert e.status == m.binding.MPCD_ENOMEM, str(e)
            failed += 1
            m.binding.debug_fail_allocs(-1)
            assert hw.current() == 0          # nothing left allocated
            continue
        m.binding.debug_fail_allocs(-1)
        s.close()
        break
    else:
        pytest.fail("create kept failing")
    assert failed >= 10                       # counters, tables, upload, slabs
    assert hw.current() == 0
    with m.Sim(pos, vel, (9, 8, 7), **kw) as s:
        s.step(2)


def _converging():
    pos, vel = workloads.fluid((12, 12, 12), 9, seed=64)
    return pos, vel - (pos - 6.0)


@pytest.mark.parametrize("prec", [m.FP32, m.FP64])
def test_failed_regrow_rolls_back_and_continues(prec):
    """Tight slabs and a converging flow: the first slab overflow needs
    larger slabs, whose allocation is made to fail. The call returns
    MPCD_ENOMEM with the state rolled back; the run then continues (a
    collision first if the failing launch was one) and ends where a run
    that never failed ends."""
    banner(f"failed regrow, prec {prec}")
    pos, vel = _converging()
    kw = dict(seed=65, precision=prec, thermostat=True, flags=m.binding.FLAG_TIGHT_SLABS)
    with m.Sim(pos, vel, (12, 12, 12), **kw) as ref:
        ref.step(6)
        want = ref.get_state()
        assert ref.layout()[3] >= 1
    with m.Sim(pos, vel, (12, 12, 12), **kw) as s:
        s.sync()
        m.binding.debug_fail_allocs(1, 1000)  # the shift table, then nothing
        with pytest.raises(m.MpcdError) as ei:
            s.step(6)
        m.binding.debug_fail_allocs(-1)
        assert ei.value.status == m.binding.MPCD_ENOMEM
        print(str(ei.value))
        done = s.step_count
        if "awaiting mpcd_collide" in str(ei.value):
            s.collide()
            done += 1
        else:
            assert "before the call" in str(ei.value) and done == 0
        s.step(6 - done)
        got = s.get_state()
    assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])


def test_readback_staging_failure():
    banner("readback staging failure")
    pos, vel = workloads.fluid((6, 6, 6), 5.0, seed=66)
    with m.Sim(pos, vel, (6, 6, 6), seed=67) as s:
        s.step(2)
        want = s.get_state()
        m.binding.debug_fail_allocs(0, 1)
        with pytest.raises(m.MpcdError) as ei:
            s.get_state()
        assert ei.value.status == m.binding.MPCD_ENOMEM
        got = s.get_state()
    assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])


def test_failed_handover_allocation_leaves_the_state_alone():
    """The solute handover's index arrays are allocated on its first use; if
    one of them cannot be, the call returns MPCD_ENOMEM having changed
    nothing, and the same call then succeeds, with the result of a run that
    never failed."""
    banner("handover allocation failure")
    pos, vel = workloads.fluid((8, 8, 8), 5.0, seed=68)
    bpos, bvel, bmass = workloads.beads((8, 8, 8), 3, 6, seed=69)
    kw = dict(seed=70, thermostat=True, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass,
              flags=m.binding.FLAG_MD_SOLUTE)
    moved = (bpos + 0.3) % 8.0

    def run(fail_at):
        with m.Sim(pos, vel, (8, 8, 8), **kw) as s:
            s.step(1)
            if fail_at is not None:
                m.binding.debug_fail_allocs(fail_at, 1)
                with pytest.raises(m.MpcdError) as ei:
                    s.set_embedded(moved, bvel)
                m.binding.debug_fail_allocs(-1)
                assert ei.value.status == m.binding.MPCD_ENOMEM
            s.set_embedded(moved, bvel)
            s.step(2)
            assert s.handover_stats() == (1, 0)
            return s.get_state()

    want = run(None)
    for k in (1, 2, 3, 4):   # the staging buffer, then the four index arrays
        got = run(k)
        assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])
