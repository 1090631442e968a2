"""Host-side checks of the Verlet-skin rebuild rule on the reference's own
reductions (no GPU): the parity cases with a skin cover both a run that
reuses one build throughout and runs that rebuild several times."""
from _parity import BuildPlan, oracles_for
import dambreak


def test_skin_schedule_exercises_both_paths():
    # the GPU skin cases: one reuses a single build for 100 steps, the others
    # rebuild several times; check that claim on the reference's reductions
    case = dambreak.make_case("c1_2d")
    counts = {}
    for skin_h in (0.3, 0.01):
        refs = oracles_for(case)
        plan = BuildPlan(skin_h * case.h)
        for r in refs:
            r.prime()
        plan.after_step(refs)
        for n in range(100):
            for r in refs:
                r.step(1)
            plan.after_step(refs)
        counts[skin_h] = plan.builds
    assert counts[0.3] == 1
    assert 3 <= counts[0.01] <= 60
