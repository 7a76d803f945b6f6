"""The oracle's pin tests against an AddressSanitizer + UndefinedBehaviorSanitizer build of the
oracle (CPU only; run.sh starts it with the sanitizer runtimes preloaded)."""
import os, shutil, sys, subprocess, tempfile
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
os.chdir(ROOT)
import oracle.oracle as O
common = ["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
tmp = tempfile.mkdtemp()
libs = (os.path.join(tmp, "oracle.so"), os.path.join(tmp, "oracle_cs.so"))
for out, extra in ((libs[0], []), (libs[1], ["-DOR_COMPLEX_STEP", "-fcx-fortran-rules"])):
    subprocess.check_call(common + extra + ["-o", out, O.SRC, "-lm"])
O.LIB, O.LIB_CS = libs
import pytest
rc = pytest.main(['-x', '-q', '-p', 'no:cacheprovider', 'tests/test_oracle_pins.py', 'tests/test_oracle_wall.py',
                  'tests/test_oracle_derivative.py'])
shutil.rmtree(tmp, ignore_errors=True)
sys.exit(rc)
