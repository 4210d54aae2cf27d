"""The pins of the default start (P13) and of the separation (P14) have teeth:
plausible mistakes planted in a copy of the oracle's functions, on the CPU, each
fail one of them.  The oracle itself is not modified."""
import inspect

import pytest

from oracle import nfhmm_oracle as O
from test_oracle_pins import check_default_start, check_separation_golden


def _mutant(fn, old, new):
    src = inspect.getsource(fn)
    assert src.count(old) == 1, f"pattern not found once in {fn.__name__}: {old!r}"
    ns = dict(vars(O))
    exec(compile(src.replace(old, new), f"<mutant of {fn.__name__}>", "exec"), ns)
    return ns[fn.__name__]


START_MUTANTS = [
    ("gamma instead of gamma/N (d-hat = 1)", "np.full((S, T, N), 1.0 / N)", "np.full((S, T, N), 1.0)"),
    ("d-hat = 1/(S N)", "np.full((S, T, N), 1.0 / N)", "np.full((S, T, N), 1.0 / (S * N))"),
    ("counts from the transposed mixture", "expected_counts(V, beta,", "expected_counts(V[::-1], beta,"),
]

SEP_MUTANTS = [
    ("source blocks swapped", "src == s] @ theta[:, src == s]", "src == S - 1 - s] @ theta[:, src == S - 1 - s]"),
    ("weights exp(E) instead of alpha / alpha_0 (reading R6)",
     "theta = alpha / alpha.sum(axis=1, keepdims=True)", "theta = np.exp(expected_log_theta(alpha))"),
    ("V instead of V / S where no source reconstructs a bin (reading R7)", "V[None] / S)", "V[None])"),
    ("state-major instead of source-major element ownership", "src, _ = element_layout(S, N, K)",
     "src = np.arange(S * N * K) % S"),
]


@pytest.mark.parametrize("name,old,new", START_MUTANTS, ids=[m[0] for m in START_MUTANTS])
def test_default_start_pin_catches(name, old, new):
    bad = _mutant(O.init_alpha, old, new)
    with pytest.raises(AssertionError):
        check_default_start(bad)


@pytest.mark.parametrize("name,old,new", SEP_MUTANTS, ids=[m[0] for m in SEP_MUTANTS])
def test_separation_pin_catches(name, old, new):
    bad = _mutant(O.separate, old, new)
    with pytest.raises(AssertionError):
        check_separation_golden(bad)


def test_unmutated_copies_pass():
    check_default_start(_mutant(O.init_alpha, "1.0 / N", "1.0 / N"))
    check_separation_golden(_mutant(O.separate, "V[None] / S)", "V[None] / S)"))
