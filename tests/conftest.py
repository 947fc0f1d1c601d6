import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


_SCENES = {}


def cached_scene(cfg: int, frame: int):
    import scenes
    key = (cfg, frame)
    if key not in _SCENES:
        _SCENES[key] = scenes.make_scene(cfg, frame)
    return _SCENES[key]


@pytest.fixture(scope="session")
def scene_cache():
    return cached_scene
