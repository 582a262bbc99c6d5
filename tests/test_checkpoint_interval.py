"""Host logic of the memory-budgeted checkpoint interval (no GPU)."""
import pytest

from paper_1607_08675_amd.adjoint import choose_interval, states_needed


def held(nsteps, k, pairs):
    """Buffers the sweep holds, counted directly: ceil(n / k) checkpoints,
    the final state and the segment states the reverse steps read (all of
    1 .. k - 1, or with paired reverse steps the even ones), or at k = 1 every
    state the sweep reads and the final one."""
    if k == 1:
        if pairs and nsteps > 1:
            return len([0] + list(range(2, nsteps, 2))) + 1
        return nsteps + 1
    seg = len(range(2, k, 2)) if pairs else k - 1
    return len(range(0, nsteps, k)) + 1 + seg


def brute_min_interval(nsteps, fit, pairs=False):
    """The smallest interval that fits; with pairs an odd one > 1 rounded up
    to the next even one, which holds no more, and that to the next multiple
    of 4 where it still fits."""
    for k in range(1, nsteps + 1):
        if held(nsteps, k, pairs) <= fit:
            if not pairs or k == 1:
                return k
            if k % 2:
                assert held(nsteps, k + 1, pairs) <= held(nsteps, k, pairs)
                k += 1
            if k % 4 and held(nsteps, k + 2, pairs) <= fit:
                k += 2
            return k
    return None


def test_everything_fits_means_no_recompute():
    assert states_needed(2000, 1) == 2001
    assert choose_interval(2000, 80 << 20, 2001 * (80 << 20)) == 1


@pytest.mark.parametrize("pairs", [False, True])
def test_matches_brute_force_over_budgets(pairs):
    for n in (1, 2, 3, 7, 50, 101, 400):
        for fit in range(2, n + 3):
            want = brute_min_interval(n, fit, pairs)
            if want is None:
                with pytest.raises(MemoryError):
                    choose_interval(n, 1000, fit * 1000, pairs)
            else:
                assert choose_interval(n, 1000, fit * 1000, pairs) == want, (n, fit)
                assert states_needed(n, want, pairs) <= fit


def test_paired_sweep_keeps_half_the_states():
    """2000 steps: every other state and the final one (1001 buffers) when
    every state the paired sweep reads is kept; with room for 161 states the
    smallest interval that fits is 13 (154 checkpoints, the final state, six
    segment states), taken as 14 (143 checkpoints, the same six) and then as
    16 (125 checkpoints, seven segment states), whose segments sweep in eight
    paired launches."""
    assert states_needed(2000, 1, True) == 1001
    assert states_needed(2000, 13, True) == 154 + 1 + 6
    assert states_needed(2000, 14, True) == 143 + 1 + 6
    assert choose_interval(2000, 1, 161, True) == 16
    assert states_needed(2000, 16, True) == 125 + 1 + 7
    # no room for the multiple of 4: stays at the even interval
    assert choose_interval(17, 1, 6, True) == 6 and states_needed(17, 8, True) > 6


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
