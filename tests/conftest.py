import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_pairsum_built():
    from oracle import pairsum
    pairsum.build(force=False)
    return True


@pytest.fixture(scope="session")
def pair001(oracle_pairsum_built):
    """Oracle problem and solve for two unit spheres at gap 0.01 moving apart
    at unit relative speed (600 proxy points, R_p = 0.7, 20 image nodes)."""
    from oracle import geometry as geo, mfs
    from paper_2407_03343_amd import workloads as wl
    pk, rbm = wl.workload_two_sphere_gap001()
    g = geo.build(pk.centers, pk.radius)
    pb = mfs.Problem(g).setup()
    out = mfs.solve_resistance(pb, rbm[0], tol=1e-10)
    return dict(pk=pk, rbm=rbm, g=g, pb=pb, out=out)


@pytest.fixture(scope="session")
def dev():
    """The HIP library's Python binding; a GPU test without a device fails
    (it does not skip), and a missing libsmfs.so raises."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    from paper_2407_03343_amd import smfs
    smfs.lib()
    return smfs
