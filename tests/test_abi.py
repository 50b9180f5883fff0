"""CPU checks of the C-ABI boundary: the library loads, exports every entry point declared in
include/afm.h, the binding's struct layouts match the header, and invalid problems are rejected
before any HIP call."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(afm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def afm():
    import paper_1109_0334_amd as afm

    if not os.path.exists(afm.LIB_PATH):
        from paper_1109_0334_amd import build

        build.build()
    return afm


def test_library_exports_every_declared_entry_point(afm):
    L = afm.lib()
    names = _declared()
    assert set(afm.EXPORTS) <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert afm.version().startswith("afm-mi355x")


_LAYOUT_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "afm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(afm_problem), offsetof(afm_problem, k),
         offsetof(afm_problem, params), offsetof(afm_problem, n_free),
         offsetof(afm_problem, lo), offsetof(afm_problem, pso_w),
         offsetof(afm_problem, polish_precision), offsetof(afm_problem, drive_mode),
         offsetof(afm_problem, steady_rtol), sizeof(afm_swarm));
  printf("%zu %zu\n", offsetof(afm_swarm, z), offsetof(afm_swarm, theta));
  return 0;
}
"""


def test_binding_struct_layout_matches_header(afm, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    src = tmp_path / "probe.c"
    src.write_text(_LAYOUT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    P, S = afm._Problem, afm._Swarm
    expect = [C.sizeof(P), P.k.offset, P.params.offset, P.n_free.offset, P.lo.offset,
              P.pso_w.offset, P.polish_precision.offset, P.drive_mode.offset,
              P.steady_rtol.offset, C.sizeof(S),
              S.z.offset, S.theta.offset]
    assert [int(x) for x in out] == expect


def _base_model():
    return dict(n_modes=1, law="dmt", k=40.0, f0=300e3, drive_freq=300e3, q=[400.0],
                ratio=[1.0], gain=[1.0], free_amplitude=20e-9, steps_per_cycle=64, n_cycles=10,
                lockin_cycles=2, ic="free_steady")


@pytest.mark.parametrize("bad", [
    dict(n_modes=0), dict(n_modes=9), dict(law=9), dict(steps_per_cycle=3),
    dict(steps_per_cycle=5000), dict(lockin_cycles=0), dict(n_cycles=1, lockin_cycles=2),
    dict(k=0.0), dict(free_amplitude=-1.0), dict(q=[0.0]), dict(ic=7), dict(drive=3),
    dict(drive="params"),  # a parameter-driven base needs ic = rest
    dict(steady_rtol=-1.0), dict(steady_rtol=float("nan")),
    dict(drive="params", ic="rest", steady_rtol=1e-6)])  # a chirp has no steady state
def test_invalid_problem_rejected_before_hip(afm, bad):
    m = dict(_base_model(), **bad)
    prob = afm.make_problem(m, [14e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9], [(1, 1e-20, 1e-19, 0)])
    h = C.c_void_p()
    code = afm.lib().afm_plan_create(C.byref(prob), 0, C.byref(h))
    assert code == 1 and not h.value
    assert afm.lib().afm_last_error().decode()


@pytest.mark.parametrize("free", [
    [(7, 0.0, 1.0, 0)], [(1, 1.0, 0.5, 0)], [(1, 0.0, 1.0, 1)], [(1, 0, 1, 0), (1, 0, 2, 0)],
    [(9, 1e3, 2e3, 0)]])  # base-motion slots are parameters only with a "params" drive
def test_invalid_search_box_rejected(afm, free):
    prob = afm.make_problem(_base_model(), [14e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9], free)
    h = C.c_void_p()
    assert afm.lib().afm_plan_create(C.byref(prob), 0, C.byref(h)) == 1


@pytest.mark.parametrize("free", [[(11, 0.0, 1.0, 0)], [(5, 0.0, 1.0, 0)],
                                  [(8, 0, 1e-9, 0), (8, 0, 2e-9, 0)]])
def test_invalid_base_motion_parameters_rejected(afm, free):
    """With a "params" drive the free slots are the law's and 8 .. 10 (a, f, g) only."""
    m = dict(_base_model(), drive="params", ic="rest")
    p = np.zeros(12)
    p[:5] = [14e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9]
    p[8:11] = [1e-9, 300e3, 0.0]
    prob = afm.make_problem(m, p, free)
    h = C.c_void_p()
    assert afm.lib().afm_plan_create(C.byref(prob), 0, C.byref(h)) == 1 and not h.value


def test_bad_precision_and_null_arguments(afm):
    prob = afm.make_problem(_base_model(), [14e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9])
    h = C.c_void_p()
    assert afm.lib().afm_plan_create(C.byref(prob), 5, C.byref(h)) == 1
    assert afm.lib().afm_plan_create(None, 0, C.byref(h)) == 1
    assert afm.lib().afm_forward_batch(None, 1, None, None, None, None, None, None, None) == 1
    assert afm.lib().afm_plan_destroy(None) == 0


def test_launch_shape_arguments_checked(afm):
    """afm_set_launch_shape validates before touching the plan (no GPU needed for the rejects)."""
    L = afm.lib()
    assert L.afm_set_launch_shape(None, 64, 1) == 1
    assert afm.lib().afm_last_error().decode()
