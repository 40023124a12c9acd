import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Tests load the oracle as built; build it only if nothing is built."""
    from oracle import _clib
    if not os.path.exists(_clib.LIB):
        _clib.build()
    yield


@pytest.fixture(autouse=True)
def _no_cone_edge_ties(request):
    """GPU parity tests: the oracle's cone-CME mask must have met no boundary
    point within its near-tie margin of the cone edge (there the kernels'
    comparison of cosines and the oracle's of arccos values may decide
    differently, which would be no error of either); fails loudly if one did."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    from oracle import boundary
    del boundary.MASK_NEAR_TIES[:]
    yield
    assert not boundary.MASK_NEAR_TIES, "cone-CME mask near-tie in the oracle: %r" % boundary.MASK_NEAR_TIES[:3]
