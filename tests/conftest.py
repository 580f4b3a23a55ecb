import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU run")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def engine():
    """One engine (context) on cuda:0 for the GPU tests; fails loudly if the
    HIP library or the GPU is missing."""
    from paper_2111_11687_amd import binding
    eng = binding.Engine(0)
    yield eng
    eng.close()


def oracle_phantom(orc, prob, activity=True):
    return orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                       [m[1] for m in prob.materials], prob.voxel_cm, label=prob.label,
                       n_organs=prob.n_organs, activity=prob.activity if activity else None)


def ledger_balance(led):
    dep = led["dep_compton"] + led["dep_pe"] + led["dep_cutoff"] + led.get("dep_positron", 0.0)
    return (dep + led["escaped"] + led["discarded"]) / led["emitted"] - 1.0
