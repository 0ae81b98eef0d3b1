"""The FP64 oracle against the paper's definitions, worked example and
proof identities, and against mathematics (closed forms, library routines,
brute force).  CPU only."""
import pytest

from oracle import bcur_oracle as O

from . import oracle_pins as P


@pytest.mark.parametrize("check", P.ALL_CHECKS, ids=lambda f: f.__name__)
def test_pin(check):
    check(O)


def test_bruteforce_all_subsets_tiny():
    errs = P.check_fit_bruteforce(O)
    assert len(errs) == 35960
