"""Host logic of the per-step cycle / lmax choice (tuning.StageSchedule and
tuning.tune_schedule) with a stand-in solver on CPU tensors: the controller's
choices follow from the recorded times alone, and the set-up search leaves the
state as it found it."""
import pytest
import torch

from paper_2011_05427_amd import tuning

V, W, F = 0, 1, 2


def test_tries_every_candidate_then_takes_the_cheapest():
    ctl = tuning.StageSchedule([(V, 1), (V, 2), (V, 4)], probe=0)
    seen = []
    for ms in (3.0, 2.0, 5.0):
        c = ctl.choose()
        seen.append(c)
        ctl.record(c, ms)
    assert seen == [(V, 1), (V, 2), (V, 4)]
    for _ in range(5):
        c = ctl.choose()
        assert c == (V, 2)
        ctl.record(c, 2.0)


def test_weighted_mean_reorders_when_the_cost_changes():
    ctl = tuning.StageSchedule([(V, 1), (W, 2)], probe=0, decay=0.5, initial={(V, 1): 1.0, (W, 2): 1.5})
    assert ctl.choose() == (V, 1)
    ctl.record((V, 1), 3.0)  # mean 0.5 * 1.0 + 0.5 * 3.0 = 2.0 > 1.5
    assert ctl.cost[(V, 1)] == pytest.approx(2.0)
    assert ctl.choose() == (W, 2)


def test_probe_reruns_the_oldest_measurement():
    ctl = tuning.StageSchedule([(V, 1), (V, 2)], probe=4, initial={(V, 1): 1.0, (V, 2): 2.0})
    choices = []
    for _ in range(9):
        c = ctl.choose()
        choices.append(c)
        ctl.record(c, 1.0 if c == (V, 1) else 2.0)
    # steps 4 and 8 probe (V, 2), whose measurement is the oldest
    assert choices == [(V, 1)] * 4 + [(V, 2)] + [(V, 1)] * 3 + [(V, 2)]


def test_ties_follow_candidate_order_and_bad_settings_are_rejected():
    ctl = tuning.StageSchedule([(F, 2), (V, 1)], probe=0, initial={(F, 2): 1.0, (V, 1): 1.0})
    assert ctl.choose() == (F, 2)
    with pytest.raises(ValueError):
        tuning.StageSchedule([])
    with pytest.raises(ValueError):
        tuning.StageSchedule([(V, 1)], decay=1.0)


class _FakeSolver:
    """Stands in for binding.Solver: a step adds lmax to T and swaps the two
    intensity buffers (as the binding does)."""

    def __init__(self):
        self.schedule = (V, 4)
        self.calls = []

    def set_schedule(self, cycle, lmax):
        self.schedule = (cycle, lmax)
        self.calls.append(("set", cycle, lmax))

    def step(self, st, **kw):
        st["T"] += self.schedule[1]
        st["I_prev"], st["I_out"] = st["I_out"], st["I_prev"]
        self.calls.append(("step",) + self.schedule)
        return None


def test_tune_schedule_restores_the_state_and_ranks_every_candidate():
    st = {"T": torch.zeros(3, dtype=torch.float64), "I_prev": torch.ones(4, dtype=torch.float64),
          "I_out": torch.full((4,), 2.0, dtype=torch.float64)}
    ref = {k: v.clone() for k, v in st.items()}
    sv = _FakeSolver()
    out = tuning.tune_schedule(sv, st, [(V, 1), (V, 2)], steps=3)
    assert set(out) == {(V, 1), (V, 2)}
    assert list(out.values()) == sorted(out.values())
    for k in ref:
        assert torch.equal(st[k], ref[k]), k
    # per candidate: two untimed steps, then the timed ones
    assert [c for c in sv.calls if c[0] == "step"].count(("step", V, 1)) == 5


def test_stage_schedule_drives_a_solver_and_records_each_step():
    st = {"T": torch.zeros(1, dtype=torch.float64), "I_prev": torch.zeros(1), "I_out": torch.zeros(1)}
    sv = _FakeSolver()
    ctl = tuning.StageSchedule([(V, 1), (V, 2)], probe=0)
    for _ in range(4):
        ctl.step(sv, st)
    assert [c for c, _ in ctl.history][:2] == [(V, 1), (V, 2)]
    assert len(ctl.history) == 4
    assert sv.calls[0] == ("set", V, 1)


def test_cost_model_follows_the_stage_without_rerunning_candidates():
    """Candidate A: one cycle per transport iteration at 1 ms; candidate B
    (W cycle through grid 2): twice the sweeps but cycles at 0.2 ms.  With
    t_sweep = 1 ms: cost_A(d) = 2 d + 1, cost_B(d) = 2.4 d + 0.2, equal at d =
    2 sweeps per step.  After both are measured, the controller keeps running
    A while the problem needs 3 sweeps per step, and switches to B when A
    itself observes 1 sweep per step (B is not re-run to learn it)."""
    A, B = ((), 1), ((2,), 1)
    ctl = tuning.CostModelSchedule([A, B], t_sweep=1.0, probe=0, decay=0.0)

    def outcome(c, d):
        s = d if c == A else 2 * d
        t = 1.0 if c == A else 0.2
        cyc = s + 1
        return s * 1.0 + cyc * t, s, cyc

    d = 3
    picks = []
    for step in range(8):
        if step == 4:
            d = 1
        c = ctl.choose()
        ms, s, cyc = outcome(c, d)
        ctl.record(c, ms, s, cyc)
        picks.append(c)
    assert picks[:2] == [A, B]  # both measured first
    assert picks[2:5] == [A, A, A]  # d = 3: A cheaper (7 vs 7.4)
    assert picks[5:] == [B, B, B]  # d = 1 seen by A: B cheaper (2.6 vs 3)
    assert ctl.predict(A) == pytest.approx(3.0) and ctl.predict(B) == pytest.approx(2.6)


def test_seeded_cost_model_starts_from_the_set_up_and_probes_near_candidates():
    """Seeded with every candidate's first 2 steps from the same state, the
    controller starts with the cheapest prediction (no order bias from the
    changing difficulty of early steps), and its periodic probes re-run only
    candidates predicted within the margin of the best."""
    A, B, C = ((), 1), ((1,), 1), ((2, 1), 1)
    # 2 steps: A 7 sweeps at 0.4 ms/cycle, B 6 sweeps at 0.45, C 6 sweeps at 2.0
    seed = {A: (7 * 1.0 + 9 * 0.4, 7, 9, 2), B: (6 * 1.0 + 8 * 0.45, 6, 8, 2), C: (6 * 1.0 + 8 * 2.0, 6, 8, 2)}
    ctl = tuning.CostModelSchedule([A, B, C], t_sweep=1.0, probe=2, decay=0.0, seed=seed, probe_margin=1.25)
    assert ctl.d == pytest.approx(3.5) and ctl.r[B] == pytest.approx(6 / 7)
    # predicted costs at d = 3.5: A 3.5 + 4.5 (9/9) 0.4 = 5.3; B 3 + 4 (8/8) 0.45 = 4.8; C 3 + 4 * 2 = 11
    assert ctl.predict(A) == pytest.approx(5.3) and ctl.predict(B) == pytest.approx(4.8)
    picks = []
    for _ in range(6):
        c = ctl.choose()
        picks.append(c)
        ms = {A: 5.3, B: 4.8, C: 11.0}[c] * 3.5 / 3.5
        s_ = {A: 3.5, B: 3.0, C: 3.0}[c]
        ctl.record(c, ms, round(s_), round(s_) + 1)
    assert picks[0] == B
    assert C not in picks  # far outside the margin: never re-run
    assert A in picks  # within 25% of the best: re-measured by a probe


def test_ratio_prior_keeps_seeded_cycle_costs_and_learns_the_ratios():
    """With a ratio prior, a candidate whose set-up steps needed more sweeps
    but whose cycles are cheaper is taken first; the recorded steps then move
    its ratio towards what it needs."""
    A, B = ((), 1), ((1,), 1)
    # set-up: A 8 sweeps at 0.4 ms per cycle, B 6 sweeps at 0.6 ms per cycle
    seed = {A: (8 * 1.0 + 10 * 0.4, 8, 10, 2), B: (6 * 1.0 + 8 * 0.6, 6, 8, 2)}
    plain = tuning.CostModelSchedule([A, B], t_sweep=1.0, probe=0, decay=0.5, seed=seed)
    # d = 4: A 4 + 5 * 0.4 = 6.0, B 3 + 4 * 0.6 = 5.4 (the set-up's ratio 6 / 8)
    assert plain.predict(A) == pytest.approx(6.0) and plain.predict(B) == pytest.approx(5.4)
    assert plain.choose() == B
    ctl = tuning.CostModelSchedule([A, B], t_sweep=1.0, probe=0, decay=0.5, seed=seed, ratio_prior=1.0)
    assert ctl.r[A] == 1.0 and ctl.r[B] == 1.0
    assert ctl.k_c[A] == pytest.approx(10 / 10) and ctl.t_c[A] == pytest.approx(0.4)
    # equal sweeps: A 4 + 5 * 0.4 = 6.0, B 4 + 5 * 0.6 = 7.0
    assert ctl.predict(B) == pytest.approx(7.0)
    assert ctl.choose() == A
    # A needs twice the sweeps that B needs at the same stage: its ratio rises
    ctl.record(B, 3 * 1.0 + 4 * 0.6, 3, 4)
    ctl.record(A, 6 * 1.0 + 7 * 0.4, 6, 7)
    assert ctl.r[A] > 1.0
    with pytest.raises(ValueError):
        tuning.CostModelSchedule([A], t_sweep=1.0, ratio_prior=0.0)


def test_cost_model_candidates_and_validation():
    ctl = tuning.CostModelSchedule([((4, 3, 2, 1), 1), (0, 2), ([1], 1)], t_sweep=0.5)
    assert ctl.cands == [((4, 3, 2, 1), 1), (0, 2), ((1,), 1)]
    with pytest.raises(ValueError):
        tuning.CostModelSchedule([], t_sweep=1.0)
    with pytest.raises(ValueError):
        tuning.CostModelSchedule([(0, 1)], t_sweep=-1.0)
    with pytest.raises(ValueError):
        tuning.CostModelSchedule([(0, 1)], t_sweep=1.0, probe_margin=0.5)
