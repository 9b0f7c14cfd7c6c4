import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a ROCm GPU (MI355X / gfx950)")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import planes
    planes._load()
    return planes


def pytest_terminal_summary(terminalreporter):
    """Report the largest GPU-versus-oracle SNR error seen, as a fraction of the tolerance."""
    mod = sys.modules.get("tests.parity")
    if mod is not None and mod.WORST["ratio"] > 0:
        terminalreporter.write_line(
            f"parity: largest SNR error {mod.WORST['ratio']:.3f} x tolerance ({mod.WORST['what']})")
