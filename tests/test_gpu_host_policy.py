"""The two execution policies of the same step bodies: the device path (HIP
kernels) and the host policy (the bodies on the host's threads) agree on
every integer bit for bit and on the FP64 state to round-off (the device
refines hardware square-root and reciprocal estimates, the host rounds
correctly)."""
import numpy as np
import pytest

import dambreak
from _parity import gpu_instance_view

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,steps", [("c1_2d", 30), ("tiny_3d", 20), ("small_batch", 10)])
def test_host_policy_equals_device_path(name, steps):
    from paper_2603_11868_amd import sph
    case = dambreak.make_case(name)
    dev = sph.Simulation(case, precision="fp64")
    host = sph.Simulation(case, precision="fp64", policy="host")
    for s in (dev, host):
        s.prime()
        s.step(steps)
    hd, hh = dev.host(), host.host()
    for b in range(len(case.instances)):
        gd, gh = gpu_instance_view(dev, hd, b), gpu_instance_view(host, hh, b)
        for k in ("key", "perm", "sorted_ids", "cell_start", "wall_start", "wall_perm", "count"):
            assert np.array_equal(gd[k], gh[k]), (b, k)
        scale_v = max(np.abs(gh["v"]).max(), 1e-30)
        assert np.abs(gd["v"] - gh["v"]).max() <= 1e-10 * scale_v, b
        assert np.abs(gd["rho"] - gh["rho"]).max() <= 1e-12 * case.rho0, b
        assert np.abs(gd["x"] - gh["x"]).max() <= 1e-12, b
        assert gd["dt"] == pytest.approx(gh["dt"], rel=1e-11)
        assert gd["diag"][12] == gh["diag"][12]          # neighbour pairs
    dev.close()
    host.close()
