"""The full-size force check's allowance for pairs at the cutoff (CPU only):
it must accept exactly the discrepancies a pair within rounding of r_c can
cause (the pair counted on one side and not on the other) and reject others."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import check_forces_at_cutoff

RC = 2.5


def _case():
    box = 10.0
    x = np.array([[2.0, 2.0], [2.0 + RC * (1 - 3e-8), 2.0], [2.0, 3.2], [7.0, 7.0]])
    md = oracle.make_md(2, len(x), box, rc=RC)
    ref, _ = oracle.forces(md, x)
    return x, box, ref


def test_pair_at_cutoff_counted_on_one_side_is_accepted():
    x, box, ref = _case()
    d = x[0] - x[1]
    term = oracle.lj_force_over_r(np.linalg.norm(d)) * d
    got = ref.copy()
    got[0] -= term      # the other side left the pair out
    got[1] += term
    n, worst = check_forces_at_cutoff(got, ref, x, x, box, RC)
    assert n == 2 and worst > 1e-4


def test_pair_just_outside_cutoff_counted_is_accepted():
    x, box, ref = _case()
    x = x.copy()
    x[1, 0] = 2.0 + RC * (1 + 3e-8)
    md = oracle.make_md(2, len(x), box, rc=RC)
    ref, _ = oracle.forces(md, x)
    d = x[0] - x[1]
    term = oracle.lj_force_over_r(np.linalg.norm(d)) * d
    got = ref.copy()
    got[0] += term      # the other side counted it
    got[1] -= term
    n, _ = check_forces_at_cutoff(got, ref, x, x, box, RC)
    assert n == 2


@pytest.mark.parametrize("which", ["no_cutoff_pair", "wrong_magnitude"])
def test_other_discrepancies_are_rejected(which):
    x, box, ref = _case()
    got = ref.copy()
    if which == "no_cutoff_pair":
        got[2] += 1e-3 * np.sqrt(np.mean(np.sum(ref ** 2, axis=1)))   # particle 2 has no pair at r_c
    else:
        d = x[0] - x[1]
        got[0] -= 2 * oracle.lj_force_over_r(np.linalg.norm(d)) * d
    with pytest.raises(AssertionError):
        check_forces_at_cutoff(got, ref, x, x, box, RC)


def test_agreeing_forces_pass_without_events():
    x, box, ref = _case()
    n, worst = check_forces_at_cutoff(ref * (1 + 1e-7), ref, x, x, box, RC)
    assert n == 0 and worst < 1e-5
