import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


class _SceneCache:
    """Full-size seeded workloads, generated once per test session (the LiDAR map takes ~30 s)."""

    def __init__(self):
        self._scenes = {}

    def get(self, name):
        if name not in self._scenes:
            import scenes
            make = {"two_view": scenes.two_view, "odometry": scenes.odometry, "lidar": scenes.lidar,
                    "dense64": scenes.dense64}[name]
            print(f"[scenes] generating {name} (seed 0, full size)", flush=True)
            self._scenes[name] = make(0)
        return self._scenes[name]


@pytest.fixture(scope="session")
def full_scenes():
    return _SceneCache()
