import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def mech_dir(tmp_path_factory):
    """The standard synthetic mechanisms written as .mech files (M9, M35, and
    the stand-ins with real-mechanism features H2R and CH4R)."""
    from chemgen.mechanism import standard_mechanism
    d = tmp_path_factory.mktemp("mech")
    for name in ("M9", "M35", "H2R", "CH4R"):
        standard_mechanism(name).write(str(d / f"{name}.mech"))
    return d


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def om9(mech_dir, oracle_lib):
    return oracle_lib.OracleMech(str(mech_dir / "M9.mech"))


@pytest.fixture(scope="session")
def om35(mech_dir, oracle_lib):
    return oracle_lib.OracleMech(str(mech_dir / "M35.mech"))
