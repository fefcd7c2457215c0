"""The C ABI without a GPU: the library loads, exports every symbol that
include/disthist.h declares, and validates arguments on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "disthist.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dh_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def dh():
    import paper_1808_01478_amd as dh
    return dh


def test_header_symbols_exported(dh):
    syms = declared_symbols()
    assert len(syms) >= 10
    lib = ctypes.CDLL(dh.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in disthist.h but not exported"
    assert sorted(dh.exported_symbols()) == syms, "binding signatures out of sync with header"


def test_strerror_and_version(dh):
    from paper_1808_01478_amd import disthist
    assert dh.version().count(".") == 2
    for code in (0, -1, -2, -3, -4, -5):
        assert disthist.LIB.dh_strerror(code)
    assert disthist.LIB.dh_strerror(-99) == b"unknown error"


ORTHO = np.diag([10.0, 11.0, 12.0])
TRIC = np.array([[10.0, 0, 0], [3.0, 9.0, 0], [-4.0, 4.0, 8.0]])


@pytest.mark.parametrize("case,expect", [
    (dict(), 0),
    (dict(r_max=0.0), -1),
    (dict(r_max=float("inf")), -1),
    (dict(r_max=float("nan")), -1),
    (dict(n_bins=0), -1),
    (dict(n_bins=1 << 24, precision=1), 0),
    (dict(n_bins=(1 << 24) + 1, precision=1), -1),
    (dict(n_bins=1 << 22), 0),                      # binary32: at most 2^22 bins
    (dict(n_bins=(1 << 22) + 1), -1),
    (dict(precision=2), -1),
    (dict(offsets=[0, 5, 3]), -1),
    (dict(offsets=[1, 5]), -1),
    (dict(offsets=[0] * 66), -1),
    (dict(box_type=3), -1),
    (dict(box_type=1, box=None), -1),
    (dict(box_type=1, box=TRIC), -1),
    (dict(box_type=1, box=np.diag([1.0, 0.0, 1.0])), -1),
    (dict(box_type=2, box=TRIC), 0),
    (dict(box_type=2, box=TRIC.T.copy()), -1),                      # upper triangular
    (dict(box_type=2, box=np.array([[10.0, 0, 0], [6.0, 9, 0], [0, 0, 8]])), -1),  # not reduced
    (dict(box_type=0, box=None), 0),
    (dict(coords_bad=True), -1),
])
def test_check_args(dh, case, expect):
    coords = np.random.default_rng(0).uniform(0, 10, size=(8, 3))
    if case.pop("coords_bad", False):
        coords[3, 1] = np.nan
    args = dict(coords=coords, offsets=[0, 5, 8], box_type=1, box=ORTHO, r_max=5.0, n_bins=10,
                precision=0)
    args.update(case)
    if args["offsets"] == [0] * 66:
        args["coords"] = None
    assert dh.check_args(**args) == expect


def test_histo_rejects_before_touching_the_device(dh):
    # invalid arguments return DH_EINVAL before any device call, so this runs
    # on a machine without a GPU
    with pytest.raises(dh.DisthistError) as e:
        dh.histo(np.zeros((4, 3)), [0, 4], 1, np.diag([1.0, -1.0, 1.0]), 0.5, 10)
    assert e.value.code == -1
    out_untouched = np.full((1, 10), 7, np.uint64)
    from paper_1808_01478_amd import disthist
    rc = disthist.LIB.dh_histo(None, np.array([0, 4], np.int64).ctypes.data_as(ctypes.c_void_p),
                               1, 0, None, 1.0, 10, 0,
                               out_untouched.ctypes.data_as(ctypes.c_void_p))
    assert rc == -1 and (out_untouched == 7).all()


def test_ctx_create_rejects_negative_budget(dh):
    # the budget is checked before the device is touched, so this runs on a
    # machine without a GPU
    from paper_1808_01478_amd import disthist
    h = ctypes.c_void_p(1)
    assert disthist.LIB.dh_ctx_create(0, -1, ctypes.byref(h)) == disthist.DH_EINVAL
    assert not h.value


def test_no_cpu_fallback_in_product_package():
    # the product package never imports the oracle
    pkg = os.path.join(ROOT, "paper_1808_01478_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.lower(), f"{f} mentions the oracle"


def test_single_hip_runtime_in_process():
    # the library must bind to the same libamdhip64 that torch uses; two
    # copies in one process leave torch unable to see the GPU
    import subprocess
    import sys
    code = ("import paper_1808_01478_amd as dh; dh.version(); import torch;"
            "m=open('/proc/self/maps').read().split('\\n');"
            "print(len(set(l.split()[-1] for l in m if 'libamdhip64' in l)))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         check=True)
    assert out.stdout.strip() == "1", out.stdout + out.stderr
