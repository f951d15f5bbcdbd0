"""Host logic of advance_to (paper_1705_00614_amd/learned.py) on a stub
solver, no GPU: it must land on the end time without passing it, also when
the CFL step grows several-fold within a run (a wet/dry front whose fastest
cell has just dried), which a cap on every step (tau_max) makes safe."""
import pytest

from paper_1705_00614_amd import learned as LC


class StubSolver:
    """Steps whose length follows `steps(k)` for step k, capped by tau_max,
    with the solver's hold_dt semantics (a held step takes the held length)."""

    def __init__(self, steps, tau_max=0.0):
        self.t, self.k, self.hold, self.tau_max = 0.0, 0, 0.0, tau_max
        self.f = steps
        self.calls = []

    def _dt(self):
        d = self.f(self.k)
        return min(d, self.tau_max) if self.tau_max > 0 else d

    def next_dt(self):
        return self.hold if self.hold > 0 else self._dt()

    def time(self):
        return self.t

    def step(self):
        self.calls.append(1)
        self.t += self.next_dt()
        self.k += 1

    def run(self, n):
        self.calls.append(n)
        for _ in range(n):
            self.t += self.next_dt()
            self.k += 1

    def hold_dt(self, d):
        self.hold = d


def jumpy(k):
    # 0.1 s for 40 steps, then 1.0 s: the step grows tenfold inside a run
    return 0.1 if k < 40 else 1.0


def test_lands_on_the_end_with_a_step_cap_when_the_step_jumps():
    for t_end in (7.9, 12.345, 100.0, 512.347):
        g = StubSolver(jumpy, tau_max=2.0)
        LC.advance_to(g, t_end)
        assert abs(g.time() - t_end) <= 1e-9 * t_end
        assert max(g.calls) <= 16


def test_without_a_cap_a_jumping_step_is_caught_not_passed_silently():
    g = StubSolver(jumpy)
    with pytest.raises(RuntimeError, match="overshot"):
        LC.advance_to(g, 10.0)


def test_without_a_cap_a_steady_step_lands():
    g = StubSolver(lambda k: 0.3)
    LC.advance_to(g, 50.0)
    assert abs(g.time() - 50.0) <= 1e-9 * 50.0


def test_already_there_takes_no_step():
    g = StubSolver(lambda k: 0.3, tau_max=1.0)
    LC.advance_to(g, 0.0)
    assert g.calls == []
