"""Host logic of bench.py's roofline models (no GPU): the method's byte floor
per beam-step, (evaluations + 1) x S with S = 2n amplitude reals, and the
whole-step fractions derived from it."""

import bench


def _form(S, amp_bytes, precision, value=1e10):
    return dict(stage_ms=[0.03] * S, n=3, amp_bytes=amp_bytes, value=value, precision=precision, beams=3200000)


def test_alg_bytes_per_beam_step():
    # Dormand-Prince with first-same-as-last: 6 new evaluations + 1 write = 7 S
    assert bench.step_roofline(_form(7, 4, 1))["alg_bytes_per_beam_step"] == 7 * 24
    assert bench.step_roofline(_form(7, 8, 0))["alg_bytes_per_beam_step"] == 7 * 48
    # classic RK4: 4 evaluations + 1 write = 5 S
    assert bench.step_roofline(_form(4, 8, 0))["alg_bytes_per_beam_step"] == 5 * 48


def test_fraction_of_the_floor():
    r = bench.step_roofline(_form(7, 4, 1, value=1e10))
    assert abs(r["frac_alg"] - 1e10 * 168 / 8e12) < 1e-4
    assert abs(r["alg_ceiling"] - 8e12 / 168) < 1.0


def test_split_error_flops_are_one_evaluation():
    # the last launch of the split Dormand-Prince error evaluates k_6 only
    f7 = bench.stage_flops(3, "dp54", 7, True)
    f1 = bench.stage_flops(3, "dp54", 1, True)
    assert f7 < f1
