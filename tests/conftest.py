import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_07441_amd import twg
    c = twg.Context(0)
    yield c
    c.close()


def scenario_tensors(sc, device="cuda"):
    """Obstacle arrays of a scenario dict as float64 device tensors."""
    import torch
    pos = torch.as_tensor(sc["pos"], dtype=torch.float64).reshape(-1, 2).contiguous().to(device)
    vel = torch.as_tensor(sc["vel"], dtype=torch.float64).reshape(-1, 2).contiguous().to(device)
    rad = torch.as_tensor(sc["rad"], dtype=torch.float64).contiguous().to(device)
    return pos, vel, rad


def reachable_scenario(name, index=0, **kw):
    """The scenario with its goal redrawn until the oracle's class map
    connects it to the start (4-neighbour flood fill)."""
    import oracle
    from paper_1903_07441_amd import scenarios
    return scenarios.reachable(
        name, index, is_reachable=lambda sc: oracle.goal_reachable(oracle.rasterize(sc)[0], sc["robot"]), **kw)
