"""The C-ABI library loads and exports every entry point include/amgs.h
declares (no device calls: this runs without a GPU)."""
import os
import re
import subprocess

from conftest import ROOT
from paper_1703_10440_amd import amgs


def header_functions():
    src = open(os.path.join(ROOT, "include", "amgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(amgs_[a-z_]+)\s*\(", src)))


def test_header_matches_binding():
    assert header_functions() == sorted(amgs.EXPORTS)


def test_library_exports_every_symbol():
    lib = amgs.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", amgs.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (amgs_\w+)", out))
    assert set(header_functions()) <= exported


def test_status_strings_and_null_handle():
    lib = amgs.load()
    assert amgs.amgs_status_string(0) == "ok"
    assert amgs.amgs_status_string(-2) == "workspace too small"
    # calls with a NULL handle fail synchronously without touching a device
    assert lib.amgs_destroy(None) == -1
    assert lib.amgs_get_stats(None, None) == -1
    assert amgs.amgs_workspace_bytes(None, 10, 2, 1, 1, 0, 0) == 0


def test_header_compiles_as_c():
    r = subprocess.run(["gcc", "-std=c99", "-fsyntax-only", "-Wall", "-Werror", "-x", "c",
                        os.path.join(ROOT, "include", "amgs.h")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_oracle_and_library_share_nothing():
    """The oracle neither includes nor loads the GPU library, and the GPU
    sources never include oracle code."""
    osrc = open(os.path.join(ROOT, "oracle", "amgs_ref.c")).read()
    assert "#include \"" not in osrc
    opy = open(os.path.join(ROOT, "oracle", "ref.py")).read()
    assert "paper_1703_10440_amd" not in opy
    csrc = os.path.join(ROOT, "paper_1703_10440_amd", "csrc")
    for f in os.listdir(csrc):
        assert "oracle" not in open(os.path.join(csrc, f)).read(), f
    for f in ("amgs.py", "build_lib.py", "__init__.py"):
        assert "oracle" not in open(os.path.join(ROOT, "paper_1703_10440_amd", f)).read(), f


def test_binding_rejects_bad_output_buffers():
    """The C ABI takes bare pointers, so the binding checks a caller's Q, P, R
    against what the kernels write before anything is launched (host tensors
    stand in for device ones: only shape, dtype, device and strides count)."""
    import pytest
    import torch
    cpu = torch.device("cpu")
    m, n = 7, 3
    good = amgs.empty_colmajor(m, n, torch.float64, cpu)
    amgs._check_out(good, "Q", m, n, torch.float64, cpu)
    padded = torch.empty((n, m + 5), dtype=torch.float64).t()[:m, :]
    amgs._check_out(padded, "Q", m, n, torch.float64, cpu)
    amgs._check_out(torch.empty(m, 1, dtype=torch.float64), "Q", m, 1, torch.float64, cpu)
    bad = [
        (amgs.empty_colmajor(m, n - 1, torch.float64, cpu), "must be 7 x 3"),     # too few columns
        (amgs.empty_colmajor(m - 1, n, torch.float64, cpu), "must be 7 x 3"),     # too few rows
        (torch.empty(m * n, dtype=torch.float64), "must be 7 x 3"),               # flat
        (amgs.empty_colmajor(m, n, torch.float32, cpu), "must be torch.float64"), # binary32 for binary64
        (torch.empty(m, n, dtype=torch.float64), "column-major"),                 # row-major
    ]
    for t, msg in bad:
        with pytest.raises(ValueError, match=msg):
            amgs._check_out(t, "Q", m, n, torch.float64, cpu)
    with pytest.raises(ValueError, match="must be on"):
        amgs._check_out(good, "Q", m, n, torch.float64, torch.device("meta"))
    with pytest.raises(ValueError, match="contiguous"):
        amgs._workspace(torch.empty(64, dtype=torch.uint8)[::2], 16, cpu)
    w = torch.empty(64, dtype=torch.uint8)
    assert amgs._workspace(w, 16, cpu) is w
