"""CPU-only checks of the C-ABI library: it loads, exports every entry point declared in include/hgks.h,
the Python binding's structures match the header, and argument validation happens on the host before
any HIP call (so these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2304_05572_amd import hgks as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgks.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hgks_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    declared = _declared_functions()
    assert set(declared) == set(H.ENTRY_POINTS)
    L = H.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_problem_struct_layout_matches_header():
    """Field order of hgks_problem / hgks_opts in the binding follows the header declaration order."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\} hgks_problem;", src, re.S).group(1)
    names = re.findall(r"([A-Za-z_][A-Za-z0-9_]*)(?:\[\d+\])?\s*[,;]", body)
    assert [f[0] for f in H.hgks_problem._fields_] == names
    body = re.search(r"typedef struct \{([^{}]*)\} hgks_opts;", src, re.S).group(1)
    names = re.findall(r"([A-Za-z_][A-Za-z0-9_]*)\s*;", body)
    assert [f[0] for f in H.hgks_opts._fields_] == names


def test_status_strings():
    for code in (H.OK, H.EINVAL, H.ENOMEM, H.EDEVICE, H.ENONPHYS, H.EDT):
        assert H.hgks_status_str(code) and H.hgks_status_str(code) != "unknown status"


@pytest.mark.parametrize("bad", [
    dict(nx=4), dict(dim=3), dict(gamma=1.0), dict(bc=(0, 1, 1, 1)), dict(dim=1, ny=3),
    dict(eqn=1, Pr=0.0), dict(recon=5), dict(cfl=0.0), dict(x1=0.0), dict(gamma_hi=1.0),
    dict(tangential_flag_mode=1),
])
def test_invalid_problems_rejected_on_host(bad):
    P = H.Problem(**bad)
    with pytest.raises(H.HgksError) as e:
        H.hgks_create([P])
    assert e.value.code == H.EINVAL


def test_mixed_dimensions_rejected():
    with pytest.raises(H.HgksError) as e:
        H.hgks_create([H.Problem(), H.Problem(dim=1, ny=1)])
    assert e.value.code == H.EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(H, "_lib", None)
    monkeypatch.setattr(H, "LIB_PATH", str(tmp_path / "libhgks.so"))
    with pytest.raises(H.HgksLibraryMissing):
        H.lib()
