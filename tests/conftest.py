import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# GPU files of the force-evaluation path run first, so that under ``-x`` a
# failure in a later addition (reaction field, Langevin, rigid water, direct
# Ewald, adjoint, batch) cannot hide them. Files not named keep their place
# after these, in collection order.
_FIRST = ("test_abi.py", "test_gpu_neighbors.py", "test_gpu_forces.py",
          "test_gpu_integrate.py")
_LAST = ("test_zz_no_alloc.py",)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(session, config, items):
    def rank(item):
        name = os.path.basename(str(item.fspath))
        if name in _FIRST:
            return _FIRST.index(name)
        if name in _LAST:
            return len(_FIRST) + 2 + _LAST.index(name)
        return len(_FIRST) + 1
    items[:] = sorted(items, key=rank)         # stable: order inside a rank is kept
