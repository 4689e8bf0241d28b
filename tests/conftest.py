import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.hookimpl(trylast=True)  # after -m deselection: only the selected tests count
def pytest_collection_modifyitems(config, items):
    # A run that selects GPU tests stops at once, with one message, when the HIP
    # library has not been built (there is no CPU path to fall back on); every
    # GPU test would otherwise fail on the same missing file.
    if any(item.get_closest_marker("gpu") for item in items):
        lib = os.path.join(ROOT, "paper_2201_00613_amd", "libsqueeze.so")
        if not os.path.exists(lib):
            pytest.exit(f"{lib} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')",
                        returncode=4)


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build()
    return oracle
