import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU oracle physics run (tens of seconds)")


def pytest_report_header(config):
    return "paper_1004_2416_amd tests (oracle pins: -m 'not gpu'; parity: -m gpu)"


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    O.lib()
    return O
