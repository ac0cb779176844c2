"""Runs the oracle through its pins with the sanitized build of the oracle's C
library (loaded through FITRIG_REF_LIB); started by tests/test_sanitizers.py
with the sanitizer runtimes preloaded."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
                      os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                      os.path.join(ROOT, "tests", "test_oracle_invariants.py")]))
