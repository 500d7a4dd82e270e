"""CPU checks of the Lambda* parity bar used by the GPU tests (tests/lstar_bar.py): it accepts
rounding-level differences and the exponent rounding its bound allows, and rejects a planted error
in a large entry, in an entry small next to its row but above 1e-30 of it, and a row-scale error."""
import numpy as np
import pytest

from lstar_bar import close_lstar


def _case(chi_value=1.0, seed=0):
    rng = np.random.default_rng(seed)
    L = rng.uniform(0.1, 1.0, (27, 4, 5, 6))
    L[3] *= 1e-20                     # entries small next to their row, still above 1e-30 of it
    L[5] *= 1e-40                     # entries below 1e-30 of their row: row-scaled bar only
    chi = np.full((4, 5, 6), chi_value)
    return L, chi


def test_accepts_rounding():
    L, chi = _case()
    close_lstar(L * (1 + 1e-14), L, chi, 8)


def test_rejects_large_entry_error():
    L, chi = _case()
    bad = L.copy()
    bad[13, 1, 2, 3] *= 1 + 1e-8
    with pytest.raises(AssertionError):
        close_lstar(bad, L, chi, 8)


def test_rejects_small_entry_error_above_threshold():
    L, chi = _case()
    bad = L.copy()
    bad[3, 2, 2, 2] *= 1 + 1e-7        # invisible to the row-scaled bar
    with pytest.raises(AssertionError):
        close_lstar(bad, L, chi, 8)


def test_ignores_entries_below_threshold_elementwise():
    L, chi = _case()
    bad = L.copy()
    bad[5] *= 2.0                      # below 1e-30 of the row: within the row-scaled bar
    close_lstar(bad, L, chi, 8)


def test_bound_grows_with_opacity():
    # a 3e-10 relative error in the entries small next to their row: within rtol + 8 eps nz chi /
    # mu_min for chi = 1e4 (nz = 4, 8 angles, mu_min ~ 0.18: 1e-10 + 3.9e-10), not for chi = 1
    L, chi = _case(chi_value=1e4)
    bad = L.copy()
    bad[3] *= 1 + 3e-10
    close_lstar(bad, L, chi, 8)
    with pytest.raises(AssertionError):
        close_lstar(bad, L, np.full_like(chi, 1.0), 8)
