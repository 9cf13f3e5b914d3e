"""tf_poisson_noalloc (static device scratch, no allocation) against tf_poisson
through the C ABI: two calls in a row on one GPU, the second on a smaller
mesh, each bitwise equal to tf_poisson on the same charges (same kernels, same
arithmetic order) and within 1e-12 of the oracle."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2602_10761_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(nx, ny, nz):
    from paper_2602_10761_amd.runtime import TriboSim
    ens = W.make_ensemble(W.CONFIGS[1].replace(nx=nx, ny=ny, nz=nz, n_particles=16, stretch=2.0, n_modes=4))
    return ens, TriboSim([ens])


def test_noalloc_poisson_equals_poisson():
    import torch
    cases = [(96, 64, 96), (24, 20, 40)]        # the second call is on a smaller mesh
    sims = [_sim(*c) for c in cases]
    for (nx, ny, nz), (ens, sim) in zip(cases, sims):
        say("noalloc poisson", (nx, ny, nz))
        g = O.Geo.from_mesh(ens.mesh)
        rng = np.random.default_rng(nx + 3 * ny)
        Q = np.zeros(g.ncell, dtype=np.int64)
        idx = rng.integers(0, g.ncell, max(8, g.ncell // 30))
        Q[idx] = rng.integers(-(1 << 50), 1 << 50, idx.size)
        q = torch.as_tensor(Q).to(sim.dev)
        phi_a = torch.full((g.ncell,), float("nan"), dtype=torch.float64, device=sim.dev)
        phi_b = torch.full((g.ncell,), float("nan"), dtype=torch.float64, device=sim.dev)
        sim.poisson_into(0, q, phi_a, noalloc=True)
        sim.poisson_into(0, q, phi_b, noalloc=False)
        sim.synchronize()
        a, b = phi_a.cpu().numpy(), phi_b.cpu().numpy()
        np.testing.assert_array_equal(a, b)
        ref = O.poisson(g, Q).ravel()
        err = np.abs(a - ref).max() / np.abs(ref).max()
        say("  rel err vs oracle", err)
        assert err < 1e-12
    for _, sim in sims:
        sim.close()


def test_noalloc_poisson_size_limit():
    from paper_2602_10761_amd.runtime import TriboError
    import torch
    # 16 * 128 * 256 * 136 bytes of spectrum: beyond the 64 MiB scratch
    ens, sim = _sim(256, 128, 256)
    n = 256 * 128 * 256
    q = torch.zeros(n, dtype=torch.int64, device=sim.dev)
    phi = torch.zeros(n, dtype=torch.float64, device=sim.dev)
    with pytest.raises(TriboError, match="TF_NOALLOC_MAX_SPECTRUM_BYTES"):
        sim.poisson_into(0, q, phi, noalloc=True)
    sim.close()
