"""sph_bind_static, the entry point for callers that cannot allocate: the
library's static device scratch in place of a caller workspace.  Two binds in
a row on one device, the second with a smaller case, each against the same
case bound with a caller workspace (sph_bind)."""
import numpy as np
import pytest

import dambreak

pytestmark = pytest.mark.gpu


def _run(case, precision, skin_h, static, steps):
    from paper_2603_11868_amd import sph
    sim = sph.Simulation(case, precision=precision, skin=skin_h * case.h, static_scratch=static)
    assert (sim.workspace is None) == static
    sim.prime()
    sim.step(steps)
    flags = sim.poll_errors()
    h = sim.host()
    builds = sim.cell_builds()
    sim.close()
    return h, flags, builds


@pytest.mark.parametrize("precision,skin_h", [("fp64", 0.0), ("mixed", 0.1)])
def test_bind_static_equals_bind(precision, skin_h):
    for name, steps in (("c1_2d", 30), ("tiny_3d", 12)):
        case = dambreak.make_case(name)
        print(f"no-alloc bind: {name} {precision} skin {skin_h} h, {steps} steps", flush=True)
        ref, f_ref, b_ref = _run(case, precision, skin_h, False, steps)
        got, f_got, b_got = _run(case, precision, skin_h, True, steps)
        assert f_ref == f_got == 0
        assert b_ref == b_got
        # the same kernels in the same order on the same inputs: identical bits
        for k in ("key", "perm", "cell_start", "wall_start", "wall_perm", "count", "id"):
            assert np.array_equal(ref[k], got[k]), (name, k)
        for k in ("x", "v", "a", "rho", "dt", "diag"):
            assert np.array_equal(ref[k], got[k]), (name, k)
