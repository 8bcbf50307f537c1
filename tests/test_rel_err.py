"""The parity metric, oracle.rel_err, against hand-computed values (CPU only).

Every GPU parity assertion compares a normwise relative error
max|y - ref| / max|ref| (the infinity norm of the difference over the
infinity norm of the reference, over the whole output tensor) with a
tolerance.  These cases fix that definition by hand: each expected value is
worked out in the comment beside it, and every case uses numbers whose
quotients are exact in binary floating point (or compares with a margin far
above rounding).  The mutants below plant plausible mistakes in copies of
the function and each must fail at least one case: a metric that always
passes would make every parity test vacuous.
"""
import inspect
import math
import textwrap

import numpy as np
import pytest

import oracle


def _case_single_element(f):
    # |1.5 - 1| / |1| = 0.5
    assert f(np.array([1.5]), np.array([1.0])) == 0.5


def _case_max_over_max(f):
    # y - ref = [0.25, 0, 2] -> max 2; max|ref| = 8 -> 0.25
    y = np.array([1.25, 8.0, -3.0])
    ref = np.array([1.0, 8.0, -5.0])
    assert f(y, ref) == 0.25


def _case_denominator_is_reference(f):
    # y - ref = [0, 2] -> max 2; max|ref| = 2 (not max|y| = 4) -> 1.0
    assert f(np.array([1.0, 4.0]), np.array([1.0, 2.0])) == 1.0


def _case_sign_mix(f):
    # y - ref = [-2, 4] -> max |.| = 4; max|ref| = 2 -> 2.0
    assert f(np.array([-1.0, 2.0]), np.array([1.0, -2.0])) == 2.0


def _case_negative_difference(f):
    # y - ref = [0, -3]: the largest error is negative; max|.| = 3, max|ref| = 1
    assert f(np.array([1.0, -2.0]), np.array([1.0, 1.0])) == 3.0


def _case_normwise_not_elementwise(f):
    # a small entry with a large relative error does not dominate:
    # max|y - ref| = 1/64 (second entry), max|ref| = 1 -> 1/64
    # (elementwise max |y - ref| / |ref| would be 1.0)
    y = np.array([1.0, 2.0 / 64.0])
    ref = np.array([1.0, 1.0 / 64.0])
    assert f(y, ref) == 1.0 / 64.0


def _case_max_not_mean(f):
    # errors [0, 0, 0, 1] -> max 1 (mean 0.25); ref magnitudes [4, 1, 1, 2]
    # -> max 4 (mean 2): 1/4 = 0.25, while a mean-based ratio is 0.125 or 0.5
    y = np.array([4.0, 1.0, -1.0, 3.0])
    ref = np.array([4.0, 1.0, -1.0, 2.0])
    assert f(y, ref) == 0.25


def _case_scale_free(f):
    # no absolute floor in the denominator: tiny outputs give the same ratio
    # as large ones (2^-40 scaling is exact)
    y = np.array([3.0, -1.0]) * 2.0 ** -40
    ref = np.array([2.0, -1.0]) * 2.0 ** -40
    assert f(y, ref) == 0.5
    assert f(y * 2.0 ** 80, ref * 2.0 ** 80) == 0.5


def _case_whole_tensor(f):
    # the max runs over every axis of the tensor, not per row:
    # row 0 error 1 with max|ref| 8, row 1 error 0 -> 1/8 (per-row max would
    # give 1/4 for row 0 if the rows' own maxima were used)
    y = np.array([[5.0, 1.0], [8.0, 0.0]])
    ref = np.array([[4.0, 1.0], [8.0, 0.0]])
    assert f(y, ref) == 0.125


def _case_zero_reference(f):
    # a nonzero output against an all-zero reference is never within tolerance
    assert f(np.array([0.0, 1e-30]), np.zeros(2)) == math.inf
    # and an all-zero output matches an all-zero reference exactly
    assert f(np.zeros(3), np.zeros(3)) == 0.0


def _case_empty(f):
    # an empty output (zero-size problem) has no error
    assert f(np.zeros(0), np.zeros(0)) == 0.0


def _case_nan_fails(f):
    # a NaN left in the output (a tile never written over a NaN sentinel) must
    # fail every `err <= tol` check
    r = f(np.array([1.0, np.nan]), np.array([1.0, 1.0]))
    assert not (r <= 1.0)


def _case_exact_match(f):
    y = np.array([[0.5, -2.0], [3.0, 1e-7]])
    assert f(y, y.copy()) == 0.0


def _case_float32_output(f):
    # outputs arrive as float32, the reference as float64: the difference is
    # taken in float64 (float32(0.1) - 0.1 = 1.49e-9, not 0)
    y = np.array([0.1], dtype=np.float32)
    r = f(y, np.array([0.1]))
    assert abs(r - abs(float(np.float32(0.1)) - 0.1) / 0.1) < 1e-12 and r > 1e-9


CASES = [_case_single_element, _case_max_over_max, _case_denominator_is_reference,
         _case_sign_mix, _case_negative_difference, _case_normwise_not_elementwise,
         _case_max_not_mean, _case_scale_free, _case_whole_tensor, _case_zero_reference,
         _case_empty, _case_nan_fails, _case_exact_match, _case_float32_output]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c.__name__[6:])
def test_rel_err(case):
    case(oracle.rel_err)


# (name, exact text in oracle.rel_err's source, replacement)
MUTANTS = [
    ("denominator_max_y", "np.max(np.abs(ref))", "np.max(np.abs(y))"),
    ("mean_numerator", "np.max(np.abs(y - ref))", "np.mean(np.abs(y - ref))"),
    ("mean_denominator", "np.max(np.abs(ref))", "np.mean(np.abs(ref))"),
    ("abs_dropped", "np.max(np.abs(y - ref))", "np.max(y - ref)"),
    ("denominator_floor", "return num / den", "return num / max(den, 1.0)"),
    ("denominator_plus_one", "return num / den", "return num / (den + 1.0)"),
    ("elementwise", "return num / den",
     "return float(np.max(np.abs(y - ref) / np.maximum(np.abs(ref), 1e-300)))"),
    ("zero_reference_passes", 'float("inf")', "0.0"),
    ("float32_difference", "y = np.asarray(y, dtype=np.float64)",
     "y = np.asarray(y); ref = np.asarray(ref, dtype=y.dtype)"),
    ("last_axis_only", "np.max(np.abs(ref))", "np.max(np.abs(ref).reshape(-1, ref.shape[-1])[0])"),
    ("nan_ignored", "np.max(np.abs(y - ref))", "np.nanmax(np.abs(y - ref))"),
]


def _mutant(old, new):
    src = textwrap.dedent(inspect.getsource(oracle.rel_err))
    assert src.count(old) >= 1, f"mutation site not found: {old}"
    ns = {"np": np}
    exec(src.replace(old, new, 1), ns)
    return ns["rel_err"]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_rel_err_mutant_fails_a_case(name, old, new):
    f = _mutant(old, new)
    failed = []
    for case in CASES:
        try:
            with np.errstate(all="ignore"):
                case(f)
        except (AssertionError, IndexError, ValueError, ZeroDivisionError):
            failed.append(case.__name__)
    assert failed, f"mutant {name} passed every case"
