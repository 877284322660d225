"""The oracle's CPU tests again, with the oracle built under AddressSanitizer
and UndefinedBehaviorSanitizer (host code only; see oracle/sanitize.py)."""
import shutil

import pytest


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_suite_under_asan_ubsan():
    from oracle import sanitize
    assert sanitize.run() == 0
