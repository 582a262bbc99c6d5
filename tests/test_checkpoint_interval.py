"""Host logic of the memory-budgeted checkpoint interval (no GPU)."""
import pytest

from paper_1607_08675_amd.adjoint import choose_interval, states_needed


def brute_min_interval(nsteps, fit):
    """Smallest k whose peak buffer count fits, by direct count of what the
    sweep holds: ceil(n / k) checkpoints, the final state and k - 1 segment
    buffers, or all n + 1 states at k = 1."""
    for k in range(1, nsteps + 1):
        held = nsteps + 1 if k == 1 else len(range(0, nsteps, k)) + 1 + (k - 1)
        if held <= fit:
            return k
    return None


def test_everything_fits_means_no_recompute():
    assert states_needed(2000, 1) == 2001
    assert choose_interval(2000, 80 << 20, 2001 * (80 << 20)) == 1


def test_matches_brute_force_over_budgets():
    for n in (1, 2, 7, 50, 101, 400):
        for fit in range(2, n + 3):
            want = brute_min_interval(n, fit)
            if want is None:
                with pytest.raises(MemoryError):
                    choose_interval(n, 1000, fit * 1000)
            else:
                assert choose_interval(n, 1000, fit * 1000) == want, (n, fit)
                assert states_needed(n, want) <= fit


def test_interval_near_square_root_when_memory_is_short():
    # 2000 steps with room for 100 states: ceil(2000/k) + k <= 100 first at k = 28
    k = choose_interval(2000, 1, 100)
    assert states_needed(2000, k) <= 100 < states_needed(2000, k - 1)
    assert 20 <= k <= 80


def test_bad_interval_rejected():
    from paper_1607_08675_amd.adjoint import Checkpointed
    for bad in (0, -3, 2.5, "every"):
        with pytest.raises(ValueError):
            Checkpointed(None, bad)
