"""CPU tests of the library boundary: symbols, host-side tree/list builders
against the oracle (integer and index results bit-exact), argument checks.
No device compute is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

mg = pytest.importorskip("paper_1609_08621_amd")


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "mgrav.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgrav_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(mg.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mg.EXPORTS)
    assert mg.version() == 3


def test_status_strings():
    for s in range(9):
        assert mg._lib.mgrav_status_string(s).decode()
    assert mg._lib.mgrav_status_string(99).decode() == "unknown status"


@pytest.fixture(scope="module")
def sets():
    return [workloads.plummer(3000, seed=21), workloads.perturbed_lattice(12, 0.2, seed=22),
            workloads.make(3, scale_n1d=16), workloads.perturbed_lattice(8, 0.0)]


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_host_tree_and_lists_equal_oracle(sets, k):
    ps = sets[k]
    to = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    tg = mg.tree_build(ps.pos, ps.mass, ps.box_L, 16)
    for f in ("perm", "cell_first", "cell_count", "child", "bucket_cell"):
        assert np.array_equal(getattr(to, f), getattr(tg, f)), f
    # the quantities that decide list membership are computed identically
    for f in ("com", "bmax", "bbox"):
        assert np.array_equal(getattr(to, f), getattr(tg, f)), f
    assert np.allclose(to.mom, tg.mom, rtol=1e-13, atol=1e-300)
    lo = oracle.build_lists(to, 0.7, ps.eps)
    lg = mg.lists_build(tg, 0.7, ps.eps)
    for f in ("pp_off", "pp_src", "pp_img", "pc_off", "pc_src", "pc_img"):
        assert np.array_equal(getattr(lo, f), getattr(lg, f)), f


def test_host_tree_rejects_bad_input():
    ps = workloads.perturbed_lattice(4, 0.1)
    with pytest.raises(mg.MgravError) as e:
        mg.tree_build(ps.pos, ps.mass, ps.box_L, 17)
    assert e.value.status == mg.ERR_INVALID_ARG
    bad = ps.pos.copy()
    bad[3, 1] = 1.5  # outside the periodic box
    with pytest.raises(mg.MgravError):
        mg.tree_build(bad, ps.mass, ps.box_L, 16)
    bad = ps.pos.copy()
    bad[0, 0] = np.nan
    with pytest.raises(mg.MgravError):
        mg.tree_build(bad, ps.mass, 0.0, 16)
    with pytest.raises(mg.MgravError):
        mg.tree_build(ps.pos, -ps.mass, ps.box_L, 16)
    t = mg.tree_build(ps.pos, ps.mass, ps.box_L, 16)
    with pytest.raises(mg.MgravError):
        mg.lists_build(t, 0.0, ps.eps)
    with pytest.raises(mg.MgravError):
        mg.lists_build(t, 0.7, ps.eps, n_images=5)


def test_workspace_size_validates_problem():
    p = mg.Problem()
    sz = ctypes.c_size_t(0)
    assert mg._lib.mgrav_workspace_size(ctypes.byref(p), ctypes.byref(sz)) == mg.ERR_INVALID_ARG
    assert b"n must be" in mg._lib.mgrav_last_error(None)
    # a plausible problem with fake (never dereferenced) device pointers
    p.n, p.eps, p.theta, p.box_L, p.n_images = 1000, 0.01, 0.7, 0.0, 1
    p.n_cell, p.n_bucket, p.n_pp, p.n_pc = 127, 64, 500, 900
    for f in ("pos", "mass", "cell_first", "cell_count", "child", "com", "bbox", "mom",
              "bucket_cell", "pp_off", "pp_src", "pp_img", "pc_off", "pc_src", "pc_img"):
        setattr(p, f, 4096)
    assert mg._lib.mgrav_workspace_size(ctypes.byref(p), ctypes.byref(sz)) == mg.OK
    assert sz.value >= 1000 * 16 + 127 * (176 + 32) + 500 * 16  # particles, cells, PP entries
    p.eps = 0.0
    assert mg._lib.mgrav_workspace_size(ctypes.byref(p), ctypes.byref(sz)) == mg.ERR_INVALID_ARG
    p.eps, p.n_images = 0.01, 27  # periodic images without a box
    assert mg._lib.mgrav_workspace_size(ctypes.byref(p), ctypes.byref(sz)) == mg.ERR_INVALID_ARG


def test_calls_on_null_context_fail_cleanly():
    assert mg._lib.mgrav_bind(None, None, None, 0) == mg.ERR_INVALID_ARG
    assert mg._lib.mgrav_compute(None, None, None) == mg.ERR_INVALID_ARG
    assert mg._lib.mgrav_wait(None, 1.0, None) == mg.ERR_INVALID_ARG
    assert mg._lib.mgrav_set_active(None, None) == mg.ERR_INVALID_ARG
    out = ctypes.c_void_p()
    assert mg._lib.mgrav_create(0, None, None) == mg.ERR_INVALID_ARG
    mg._lib.mgrav_destroy(None)


def test_interact_variants_and_their_argument_checks():
    v = mg.interact_variants()
    assert len(v) >= 2 and v[0] == (48, 3, 0)
    for chunk, waves, prefetch in v:
        assert 1 <= chunk <= 64 and 1 <= waves <= 8 and prefetch in (0, 1)
        assert not prefetch or waves <= 2  # the prefetch needs the 2-wave register budget
    assert len(set(v)) == len(v)
    ch = ctypes.c_int(0)
    assert mg._lib.mgrav_interact_variant_info(len(v), ctypes.byref(ch), None,
                                               None) == mg.ERR_INVALID_ARG
    assert mg._lib.mgrav_interact_variant_info(-1, None, None, None) == mg.ERR_INVALID_ARG
    assert mg._lib.mgrav_interact_variants(None) == mg.ERR_INVALID_ARG
    assert mg._lib.mgrav_set_interact_variant(None, 0) == mg.ERR_INVALID_ARG
    assert mg._lib.mgrav_autotune(None, None, None, None, 100.0, None, None) == mg.ERR_INVALID_ARG


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct (checked with gcc)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pairs = [("mgrav_problem", mg.Problem), ("mgrav_ewald", mg.EwaldConfig),
             ("mgrav_stats", mg.Stats), ("mgrav_train_cfg", mg.TrainConfig),
             ("mgrav_tree_dev", mg.TreeDev), ("mgrav_walk", mg.Walk), ("mgrav_store", mg.Store),
             ("mgrav_fmm", mg.Fmm)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mgrav.h"',
             "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        cname, key, val = ln.split()
        got[(cname, key)] = int(val)
    for cname, cls in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_watchdog_times_out_on_a_query_that_never_completes():
    """The wait policy against a fake completion query that never reports
    done (the paper's GPU that accepts work and never finishes it, Appendix
    A): TIMEOUT after the deadline, not before; completion after a few
    polls returns OK; a failing query returns DEVICE at once."""
    import time
    polls = []

    def never():
        polls.append(1)
        return 1

    t0 = time.perf_counter()
    st = mg.watchdog_poll(never, 0.05)
    dt = time.perf_counter() - t0
    assert st == mg.ERR_TIMEOUT
    assert 0.05 <= dt < 1.0 and len(polls) > 3
    assert "deadline" in mg._lib.mgrav_last_error(None).decode()

    count = iter(range(5, -1, -1))
    assert mg.watchdog_poll(lambda: next(count), 5.0) == mg.OK

    assert mg.watchdog_poll(lambda: -1, 5.0) == mg.ERR_DEVICE
    assert mg._lib.mgrav_watchdog_poll(mg.WATCHDOG_QUERY(), None, 1.0) == mg.ERR_INVALID_ARG


def test_integrator_schedule_matches_the_oracle():
    """The device integrator's host-side schedule (which rungs end a step at
    each substep boundary) is the oracle's."""
    from oracle import kdk
    from paper_1609_08621_amd import kdk as dkdk
    for R in range(0, 7):
        assert [dkdk.boundary_rung(k, R) for k in range((1 << R) + 1)] == \
            [kdk.boundary_rung(k, R) for k in range((1 << R) + 1)]


def test_store_calls_refuse_bad_arguments_on_the_host():
    st = mg.Store()
    assert mg._lib.mgrav_store_encode(None, 10, None, None, 1, ctypes.byref(st)) == \
        mg.ERR_INVALID_ARG
    assert mg._lib.mgrav_store_drift(None, 10, ctypes.byref(st), 0.1, 1) == mg.ERR_INVALID_ARG


@pytest.mark.parametrize("k", [0, 1, 2])
def test_host_fmm_lists_equal_oracle(sets, k):
    """The library's fast-multipole walk (C++, tasks over subtrees) gives the
    oracle's lists entry for entry."""
    ps = sets[k]
    t = mg.tree_build(ps.pos, ps.mass, ps.box_L, 16)
    pt = ps.pos[t.perm]
    lg = mg.fmm_lists_build(t, pt, 0.7, ps.eps)
    to = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    lo = oracle.build_fmm_lists(to, pt, 0.7, ps.eps)
    for f in ("pp_off", "pp_src", "pp_img", "pp_sub", "pc_off", "pc_src", "pc_img", "cc_off",
              "cc_src", "cc_img"):
        assert np.array_equal(getattr(lg, f), getattr(lo, f)), f
    assert lo.cc_src.size > 0 and (lo.cc_src < 0).any() and (lo.pp_sub > 0).any()


def test_import_fails_loudly_without_the_library(tmp_path):
    """No CPU fallback: with the HIP library absent the binding does not import."""
    import subprocess
    import sys
    env = dict(os.environ, MGRAV_LIBRARY=str(tmp_path / "libmgrav_absent.so"))
    r = subprocess.run([sys.executable, "-c", "import paper_1609_08621_amd"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "no fallback" in r.stderr
