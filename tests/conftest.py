"""Shared fixtures: builds of the oracle and the input generator, the gpu marker."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libs():
    import oracle
    from paper_1803_01112_amd import synth
    oracle.build(force=False)
    synth.build(force=False)
