"""Host logic: when the optimisation loop evaluates the learned guess."""
from paper_2210_00947_amd.topopt import GuessSchedule


def run(s, outcomes, n):
    """Evaluate on the cycles the schedule asks for; outcomes[i] is whether
    the i-th evaluation wins. Returns the evaluated cycle indices."""
    seen, it = [], iter(outcomes)
    for c in range(n):
        if s.want():
            seen.append(c)
            s.record(next(it))
    return seen


def test_losses_back_off_doubling_to_the_cap():
    # losses on every evaluation: gaps 1, 2, 4, 8, then 8 (cap) cycles
    assert run(GuessSchedule(cap=8), [False] * 20, 60) == [0, 2, 5, 10, 19, 28, 37, 46, 55]


def test_a_win_resets_the_gap():
    # lose, lose (gap 2 next), win (reset), lose (gap 1 next), ...
    seen = run(GuessSchedule(cap=16), [False, False, True, False, True, True], 10)
    assert seen == [0, 2, 5, 6, 8, 9]


def test_disabled_evaluates_every_cycle():
    assert run(GuessSchedule(enabled=False), [False] * 10, 10) == list(range(10))
