import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import ftlm as of
    return of.lib()


@pytest.fixture
def force_variant(monkeypatch):
    """force_variant(variant, kc=0): every Hamiltonian the test creates gets
    this H*v launch for both precisions and every column count, through the
    C ABI's tuning call (ftlm_hamiltonian_set_tuning)."""
    def apply(variant, kc=0):
        import paper_2607_25585_amd as F
        orig = F.Hamiltonian.__init__

        def init(self, system, _orig=orig):
            _orig(self, system)
            for prec in (F.FTLM_C128, F.FTLM_C64):
                for k in range(1, 65):
                    self.set_tuning(prec, k, int(variant), 0, int(kc))
        monkeypatch.setattr(F.Hamiltonian, "__init__", init)
    return apply


@pytest.fixture
def plan_windows():
    """plan_windows(pass_kb=0, l2_kb=0, tile_kb=0): window sizes of the H*v
    planners for the Hamiltonians the test creates afterwards (through the C
    ABI's ftlm_set_plan_windows); the defaults are restored after the test."""
    import paper_2607_25585_amd as F

    def apply(pass_kb=0, l2_kb=0, tile_kb=0):
        F.set_plan_windows(pass_kb, l2_kb, tile_kb)
    yield apply
    F.set_plan_windows(0, 0, 0)
