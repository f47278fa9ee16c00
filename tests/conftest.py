import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def full_hp():
    from paper_2604_24816_amd import inputs
    return inputs.FULL_HPARAMS


@pytest.fixture(scope="session")
def full_model(full_hp):
    import oracle
    from paper_2604_24816_amd import inputs
    return oracle.Model.from_hparams(full_hp, inputs.random_model(full_hp, 0))
