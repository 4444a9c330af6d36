import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


@pytest.fixture(scope="session")
def mech_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("mech"))


@pytest.fixture(scope="session")
def small(mech_dir):
    from paper_2205_05681_amd import synth
    import oracle
    path, m = synth.mechanism_file("small", mech_dir)
    return path, m, oracle.Oracle(path)


@pytest.fixture(scope="session")
def ch4(mech_dir):
    from paper_2205_05681_amd import synth
    import oracle
    path, m = synth.mechanism_file("ch4", mech_dir)
    return path, m, oracle.Oracle(path)


@pytest.fixture(scope="session")
def large(mech_dir):
    from paper_2205_05681_amd import synth
    import oracle
    path, m = synth.mechanism_file("large", mech_dir)
    return path, m, oracle.Oracle(path)
