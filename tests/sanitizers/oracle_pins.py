"""The oracle's pin tests against a sanitized build of the oracle library
(argv[1]); run by run.sh with the sanitizer runtimes preloaded."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

oracle._LIB_PATH = sys.argv[1]
oracle.build = lambda force=True: oracle._LIB_PATH
import pytest  # noqa: E402

sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", os.path.join(ROOT, "tests", "test_oracle_pins.py")]))
