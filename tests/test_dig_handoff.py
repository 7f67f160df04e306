"""The DIG driver's hand-off rule (host logic, no GPU): DIG guidance stops
once the cycle-to-cycle change of the macroscopic solution has levelled off,
i.e. its mean over the last window is above `handoff` times the mean over
the window before."""
import types

from paper_2501_10965_amd.dig import DIG


def _driver(changes, handoff=0.95):
    return types.SimpleNamespace(log=[{"cycle": k, "cycle_change": c}
                                      for k, c in enumerate(changes)],
                                 handoff=handoff, HANDOFF_WINDOW=DIG.HANDOFF_WINDOW)


def test_no_decision_before_two_windows():
    n = DIG.HANDOFF_WINDOW
    assert not DIG._levelled_off(_driver([0.2] * (2 * n - 1)))
    assert DIG._levelled_off(_driver([0.2] * (2 * n)))


def test_falling_change_keeps_guiding():
    n = DIG.HANDOFF_WINDOW
    falling = [0.5 * 0.97 ** k for k in range(2 * n)]  # 26 % lower per window
    assert not DIG._levelled_off(_driver(falling))


def test_noise_plateau_hands_off():
    n = DIG.HANDOFF_WINDOW
    plateau = [0.16 + 0.004 * ((-1) ** k) for k in range(2 * n)]
    assert DIG._levelled_off(_driver(plateau))
    # a threshold of 1.0 needs the change to grow
    assert not DIG._levelled_off(_driver([0.2] * n + [0.19] * n, handoff=1.0))


def test_cycles_without_a_solve_are_ignored():
    n = DIG.HANDOFF_WINDOW
    log = _driver([0.2] * (2 * n))
    log.log.insert(3, {"cycle": 99})  # a plain DSMC cycle: no change recorded
    assert DIG._levelled_off(log)
