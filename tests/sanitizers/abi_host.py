"""The C-ABI host tests against a copy of the binding (argv[1]) whose
libmcspect has sanitized host code; run by run.sh with the runtime preloaded."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, sys.argv[1])
sys.path.insert(1, ROOT)
import paper_2105_13324_amd as mc  # noqa: E402

assert mc.LIB_PATH.startswith(sys.argv[1]), mc.LIB_PATH
import pytest  # noqa: E402

sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", os.path.join(ROOT, "tests", "test_abi_host.py")]))
