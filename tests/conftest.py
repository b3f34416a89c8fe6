import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_CONFIG = None


def pytest_configure(config):
    global _CONFIG
    _CONFIG = config
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def say(msg: str) -> None:
    """Print a progress line of a long test straight to the terminal, past
    pytest's output capture (what capsys.disabled() does), so a run of
    several minutes shows which step it is in."""
    capman = _CONFIG.pluginmanager.getplugin("capturemanager") if _CONFIG is not None else None
    if capman is None:
        print(msg, flush=True)
        return
    with capman.global_and_fixture_disabled():
        print(msg, flush=True)


_CACHE = {}


def cached(key, fn):
    """Process-wide cache for generated matrices shared between tests."""
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]
