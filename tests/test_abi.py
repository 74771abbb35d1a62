"""C-ABI contract checks that need no GPU: the library loads, it exports every
function include/sgs.h declares, and host-side validation rejects bad input."""

import ctypes
import os
import re

import numpy as np
import pytest

import sgs_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgs.h")
LIB = os.path.join(ROOT, "paper_2105_01088_amd", "libsgs.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsgs.so not built")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sgs_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2105_01088_amd import load_library
    lib = load_library()
    names = _declared()
    assert "sgs_step" in names and "sgs_init" in names and len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_one_hip_runtime_per_process():
    """Loading the library must not bring in a second HIP runtime beside
    torch's (two runtimes in one process leave torch without a GPU)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); from paper_2105_01088_amd._lib import load_library; "
            "load_library(); import torch; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_default_options():
    from paper_2105_01088_amd import default_options, SGS_FP64, SGS_W_PRINTED
    o = default_options()
    assert o.precision == SGS_FP64 and o.weight == SGS_W_PRINTED
    assert o.g_rel_threshold == 1e-12 and o.purify_iters >= 3
    assert o.update == 0 and o.exp_coef == 0.25  # Euler + purification; App. A coefficient read as 1/4


def test_default_options_rejects_unknown_fields():
    """A misspelt option must not be dropped silently by the ctypes mirror."""
    from paper_2105_01088_amd import default_options
    with pytest.raises(TypeError):
        default_options(stream=2)


def _ws(ham, R, **opt):
    from paper_2105_01088_amd._lib import _HostProblem, default_options, load_library, sgs_problem
    lib = load_library()
    hp = _HostProblem(ham, R)
    arr = (sgs_problem * 1)(hp.s)
    o = default_options(**opt)
    nb = ctypes.c_size_t(0)
    rc = lib.sgs_workspace_bytes(arr, 1, ctypes.byref(o), ctypes.byref(nb))
    return rc, nb.value


def test_workspace_size_scales_with_pairs():
    ham = si.anderson(7, 1.0, 0.5)
    rc1, b1 = _ws(ham, 4)
    rc2, b2 = _ws(ham, 8)
    assert rc1 == 0 and rc2 == 0
    assert b2 > b1 > 8 * 4 * 32 * 32


def test_rejects_bad_problems_and_options():
    ham = si.anderson(3, 1.0, 0.5)
    assert _ws(ham, 0)[0] == -1          # R out of range
    assert _ws(ham, 33)[0] == -1
    bad = si.anderson(3, 1.0, 0.5)
    bad.A = bad.A.copy()
    bad.A[0, 5] += 1.0                   # not skew
    assert _ws(bad, 2)[0] == -1
    bad2 = si.anderson(3, 1.0, 0.5)
    bad2.quartic_idx = np.array([[0, 2, 1, 3]], dtype=np.int32)  # not increasing
    assert _ws(bad2, 2)[0] == -1
    bad3 = si.anderson(3, 1.0, 0.5)
    bad3.quartic_idx = np.array([[0, 1, 2, 999]], dtype=np.int32)  # out of range
    assert _ws(bad3, 2)[0] == -1
    assert _ws(ham, 2, weight=7)[0] == -1
    assert _ws(ham, 2, precision=5)[0] == -1
    assert _ws(ham, 2, purify_iters=0)[0] == -1
    assert _ws(ham, 2, update=2)[0] == -1
    assert _ws(ham, 2, update=1, exp_coef=0.0)[0] == -1
    assert _ws(ham, 2, update=1, exp_coef=float("nan"))[0] == -1


def test_exponential_map_workspace():
    """The exponential map carves four more R n^2 buffers, the n R row sums
    and its job tables; the Euler workspace is unchanged by the option's
    existence."""
    ham = si.anderson(7, 1.0, 0.5)
    rc0, b0 = _ws(ham, 4)
    rc1, b1 = _ws(ham, 4, update=1)
    assert rc0 == 0 and rc1 == 0
    n = ham.n
    assert b1 - b0 >= 4 * 4 * n * n * 8


def test_strerror_and_null_context():
    from paper_2105_01088_amd import load_library
    lib = load_library()
    assert lib.sgs_strerror(0) == b"ok"
    assert b"workspace" in lib.sgs_strerror(-9)
    assert b"exponential" in lib.sgs_strerror(-10)
    assert lib.sgs_step(None, 0.05, 1, None) == -1
    assert lib.sgs_pair_eval(None, None, None, None, None) == -1
    assert lib.sgs_energy(None, None, None) == -1
