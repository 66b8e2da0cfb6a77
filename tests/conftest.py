import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def water_oracle():
    from oracle import Oracle
    from paper_2304_09409_amd import synth
    return Oracle(synth.WATER_MODEL, synth.water_params())


@pytest.fixture(scope="session")
def serve_oracle():
    from oracle import Oracle
    from paper_2304_09409_amd import synth
    return Oracle(synth.SERVE_MODEL, synth.serve_params())


@pytest.fixture(scope="session")
def fcc_oracle():
    from oracle import Oracle
    from paper_2304_09409_amd import synth
    return Oracle(synth.FCC_MODEL, synth.fcc_params())
