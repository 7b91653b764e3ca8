"""The synchronous step calls replay a graph of 32 attempts captured on the
run's stream; with kernel timing on (or fewer than 32 attempts) they launch
every attempt directly.  Both orders of the same kernels give the same bits:
states, phases and counters after two calls that each mix graph replays and
direct launches.  Also the small adaptive run of the 2-flavor single-angle
physics, in which launch overhead dominates, against its direct twin."""

import sys

import numpy as np
import pytest

from paper_1907_05560_amd import nuosc, workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _twin_runs(w, calls):
    with nuosc.Run(w) as a, nuosc.Run(w) as b:
        b.timing_enable(True)  # direct launches throughout
        for n in calls:
            a.step(n)
            b.step(n)
        pa, fa = a.get_state()
        pb, fb = b.get_state()
        sa, sb = a.stats(), b.stats()
    return (pa, fa, sa), (pb, fb, sb)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_AMP])
def test_graph_replayed_attempts_equal_direct_launches(prec):
    w = W.multi_angle_3f(37, 13)
    w.update(precision=prec)
    say(f"case: graph replay vs direct launches, 3f 37x13, prec={prec}")
    # 70 = two replays and 6 direct, 45 = one replay and 13 direct
    (pa, fa, sa), (pb, fb, sb) = _twin_runs(w, (70, 45))
    np.testing.assert_array_equal(pa, pb)
    np.testing.assert_array_equal(fa, fb)
    assert sa == sb, (sa, sb)
    assert sa["accepted"] + sa["rejected"] == 115


def test_graph_replay_on_the_single_angle_rk4_run():
    # started at 50 km, where the explicit fixed step is stable
    w = W.single_angle_2f()
    w["r_start_km"] = 50.0
    say("case: graph replay vs direct launches, 2f single-angle RK4 from 50 km")
    (pa, fa, sa), (pb, fb, sb) = _twin_runs(w, (200,))
    np.testing.assert_array_equal(pa, pb)
    np.testing.assert_array_equal(fa, fb)
    assert sa == sb and sa["accepted"] == 200, (sa, sb)
