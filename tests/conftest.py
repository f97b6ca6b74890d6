import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def wind_large_ref(oracle_mod):
    """The 1024 x 2048 wind workload (3 fields, 2,097,152 points) with the
    oracle on its 10^4 sampled points (default_rng(15), without
    replacement): (workload, sample indices, oracle values [3][10^4])."""
    import synth
    wl = synth.workload_large()
    idx = synth.sample_indices(wl.n_pts, 10000, seed=15)
    ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi[idx], wl.theta[idx])
    return wl, idx, ref


@pytest.fixture(scope="session")
def sbr_full_ref(oracle_mod):
    """The 256 x 512 solid-body-rotation workload (3 fields, 131,072 points)
    with the oracle at every point: (workload, oracle values [3][131072])."""
    import synth
    wl = synth.workload_sbr()
    return wl, oracle_mod.dfs_eval(wl.coeffs, wl.phi, wl.theta)
