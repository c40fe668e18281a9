"""pytest plugin of the sanitizer runs (tests/test_sanitizers.py): points the
device library's binding (CM_SANITIZED_LIB) or the oracle (ORACLE_SANITIZED_LIB)
at a build instrumented with AddressSanitizer and UndefinedBehaviorSanitizer,
before any test loads it."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

if os.environ.get("CM_SANITIZED_LIB"):
    from paper_2003_03130_amd import _native
    _native.LIB_PATH = os.environ["CM_SANITIZED_LIB"]
if os.environ.get("ORACLE_SANITIZED_LIB"):
    import oracle
    oracle._SO = os.environ["ORACLE_SANITIZED_LIB"]
