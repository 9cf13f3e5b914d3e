"""Per-phase timing through the C ABI: events bracket the requested phases of
the requested steps and leave the results unchanged."""
import sys

import numpy as np
import pytest

from helpers import KEYS
from paper_2602_10761_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_profile_phases_and_stride():
    from paper_2602_10761_amd.runtime import PHASES, TriboSim
    spec = W.CONFIGS[1].replace(nx=32, ny=32, nz=32, n_particles=5000, v_jitter=2.0, precharge=0.2)
    ens = W.make_ensemble(spec, 1, 0)
    say("profile all phases, then every 3rd step")
    sim = TriboSim([ens])
    sim.step(1)
    sim.profile_begin(3)
    sim.step(3)
    ms, n = sim.profile_end()
    assert n == 3
    for p in ("deposit_fftx", "fftz_fwd", "tridiag", "fftz_inv", "push"):
        assert ms[p] > 0.0, p
    assert all(v >= 0.0 for v in ms.values())
    sim.profile_begin(2, phases=["push"], every=3)
    sim.step(6)
    ms2, n2 = sim.profile_end()
    assert n2 == 2
    assert ms2["push"] > 0.0
    assert all(v == 0.0 for k, v in ms2.items() if k != "push")
    prof = sim.state_np(0)
    from paper_2602_10761_amd.runtime import TriboError
    with pytest.raises(TriboError, match="every"):
        sim.profile_begin(2, every=0)
    sim.close()
    plain = TriboSim([ens])
    plain.step(10)
    ref = plain.state_np(0)
    plain.close()
    for k in KEYS:
        np.testing.assert_array_equal(prof[k], ref[k])
    say("  ok", {k: round(v, 4) for k, v in ms.items()})
