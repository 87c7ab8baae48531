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
    return sorted(set(re.findall(r"\b(hgks_[a-z0-9_]+)\s*\(", src)))


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


def test_bc_data_layout_matches_header():
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\} hgks_bc_data;", src, re.S).group(1)
    names = re.findall(r"([A-Za-z_][A-Za-z0-9_]*)(?:\[\d+\])?\s*[,;]", body)
    assert [f[0] for f in H.hgks_bc_data._fields_] == names
    assert C.sizeof(H.hgks_bc_data) == 8 * 11 + 8


def test_stepper_layout_matches_header():
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\} hgks_stepper;", src, re.S).group(1)
    names = re.findall(r"([A-Za-z_][A-Za-z0-9_]*)(?:\[\d+\])*\s*[,;]", body)
    assert [f[0] for f in H.hgks_stepper._fields_] == names
    assert C.sizeof(H.hgks_stepper) == 8 + 8 * (9 + 9 + 3 + 3)


def test_status_strings():
    for code in (H.OK, H.EINVAL, H.ENOMEM, H.EDEVICE, H.ENONPHYS, H.EDT):
        assert H.hgks_status_str(code) and H.hgks_status_str(code) != "unknown status"


@pytest.mark.parametrize("bad", [
    dict(nx=4), dict(dim=3), dict(gamma=1.0), dict(bc=(0, 1, 1, 1)), dict(dim=1, ny=3),
    dict(eqn=1, Pr=0.0), dict(recon=5), dict(cfl=0.0), dict(x1=0.0), dict(gamma_hi=1.0),
    dict(tangential_flag_mode=2), dict(dim=1, ny=1, tangential_flag_mode=1), dict(positivity=2),
    dict(dim=3, nz=8, tangential_flag_mode=1),
    dict(char_state_mode=2), dict(dim=1, ny=1, char_state_mode=1), dict(dim=3, nz=8, char_state_mode=1),
    dict(viscous_dt_mode=2), dict(dim=3, nz=8, viscous_dt_mode=-1),
    # prescribed-state sides: no data (rest 0), a periodic rest, NaN split, non-physical states
    dict(bc=(4, 1, 1, 1)), dict(bc=(4, 1, 1, 1), bcd=(H.BcData(rest=0),)),
    dict(bc=(0, 4, 1, 1), bcd=(None, H.BcData())),
    dict(bc=(1, 1, 4, 1), bcd=(None, None, H.BcData(s0=float("nan")))),
    dict(bc=(1, 1, 1, 4), bcd=(None, None, None, H.BcData(st=float("inf")))),
    dict(bc=(4, 1, 1, 1), bcd=(H.BcData(a=(1.0, 0.0, 0.0, -1.0)),)),
    dict(bc=(4, 1, 1, 1), bcd=(H.BcData(b=(-1.0, 0.0, 0.0, 2.5)),)),
    dict(dim=1, ny=1, bc=(1, 4, 0, 0), bcd=(None, H.BcData(a=(1.0, 3.0, 0.0, 1.0), rest=2))),
    # three dimensions: too few z cells, unpaired or unknown z sides, what the 3D path does not take
    dict(dim=3, nz=4), dict(dim=3, nz=8, bcz=(0, 1)), dict(dim=3, nz=8, bcz=(1, 4)), dict(dim=3, nz=8, z1=0.0),
    dict(dim=3, nz=8, eqn=1, mu=1e-3, Pr=0.72), dict(dim=3, nz=8, positivity=1),
    dict(dim=3, nz=8, bc=(4, 1, 1, 1), bcd=(H.BcData(),)),
    # multistage tableaux: stage count, non-finite coefficients, what only S2O4 supports
    dict(stepper=H.Stepper(4, b=(1, 0, 0))), dict(stepper=H.Stepper(-1)),
    dict(stepper=H.Stepper(1, b=(1, 0, 0), bh=(float("nan"), 0, 0))),
    dict(stepper=H.Stepper(2, a=((0, 0, 0), (float("inf"), 0, 0), (0, 0, 0)), b=(1, 0, 0))),
    dict(stepper=H.Stepper(1, b=(1, 0, 0), bh=(0.5, 0, 0)), positivity=1),
    dict(stepper=H.Stepper(1, b=(1, 0, 0), bh=(0.5, 0, 0)), bc=(4, 1, 1, 1), bcd=(H.BcData(),)),
])
def test_invalid_problems_rejected_on_host(bad):
    P = H.Problem(**bad)
    with pytest.raises(H.HgksError) as e:
        H.hgks_create([P])
    assert e.value.code == H.EINVAL


def test_compensated_accumulation_rejected_in_3d():
    with pytest.raises(H.HgksError) as e:
        H.hgks_create([H.Problem(dim=3, nx=8, ny=8, nz=8)], compensated=1)
    assert e.value.code == H.EINVAL


def test_mixed_steppers_and_compensated_tableau_rejected():
    one = H.Stepper(1, b=(1, 0, 0), bh=(0.5, 0, 0))
    with pytest.raises(H.HgksError) as e:
        H.hgks_create([H.Problem(), H.Problem(stepper=one)])
    assert e.value.code == H.EINVAL
    with pytest.raises(H.HgksError) as e:
        H.hgks_create([H.Problem(stepper=one)], compensated=1)
    assert e.value.code == H.EINVAL


def test_mixed_tangential_flag_modes_rejected():
    with pytest.raises(H.HgksError) as e:
        H.hgks_create([H.Problem(), H.Problem(tangential_flag_mode=1)])
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


C_EXAMPLE = r"""
#include <stdint.h>
#include "hgks.h"
/* the usage example of the README: the header is plain C and the documented calls type-check */
int run_example(const double* W0, double* W) {
  hgks_problem p = {.dim = 2, .nx = 1024, .ny = 1024, .x1 = 1, .y1 = 1, .eqn = HGKS_EULER, .gamma = 1.4,
                    .Pr = 1, .cfl = 0.5, .c1 = 0.01, .c2 = 1, .bc = {1, 1, 1, 1}, .recon = HGKS_RECON_HYBRID,
                    .gamma_hi = 0.85, .gamma_lo = 0.85, .weno_eps = 1e-8};
  hgks_opts o = {.precision = HGKS_FP64, .autotune = 1, .use_graph = 1, .tile = -1};
  hgks_t* h;
  double t = 0.0, t_end = 0.25;
  int32_t tile[5];
  double prof[8];
  if (hgks_create(&p, 1, &o, &h) != HGKS_OK) return 1;
  hgks_set_ic(h, 0, W0, 0, 0.0);
  hgks_run(h, &t_end, INT64_MAX, NULL);
  hgks_get_state(h, 0, W, 0, &t);
  hgks_get_state_lo(h, 0, W, 0);
  hgks_get_tile(h, tile);
  hgks_get_profile(h, prof);
  hgks_destroy(h);
  return (int)hgks_status_str(HGKS_OK)[0] + HGKS_NUM_LAUNCH_CONFIGS;
}
"""


def test_header_is_plain_c_and_the_readme_example_compiles(tmp_path):
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "example.c"
    src.write_text(C_EXAMPLE)
    r = subprocess.run([cc, "-std=c11", "-Wall", "-Werror", "-pedantic", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_launch_config_count_matches_binding():
    src = open(HEADER).read()
    m = re.search(r"#define HGKS_NUM_LAUNCH_CONFIGS (\d+)", src)
    assert m and int(m.group(1)) == H.NUM_LAUNCH_CONFIGS
