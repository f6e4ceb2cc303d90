"""The C-ABI library loads and exports every symbol the header declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polyreact.h")
LIB = os.path.join(ROOT, "paper_1409_7498_amd", "libpolyreact.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1409_7498_amd.csrc import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared()
    for n in ("pr_react_step", "pr_sys_create", "pr_sys_run", "pr_sys_bonds", "pr_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1409_7498_amd import binding
    assert set(binding.exported_symbols()) <= set(declared())


def test_host_validation_without_gpu():
    """Argument errors are reported before any device call."""
    from paper_1409_7498_amd import binding as b
    r = b.Rule.make(type_a=1, a_min=1, a_max=4, d_a=-1, type_t=0, t_min=1, t_max=2, d_t=-1,
                    rc=1.12, exclude_bonded=1, p=0.5)
    nb = ctypes.c_int32(0)
    st = b.Stats()
    L = ctypes.c_float(2.0)  # L <= 2 rc
    code = b.lib.pr_react_step(10, L, None, None, None, None, None, None, 4, ctypes.byref(r), 1, 1,
                               None, 5, ctypes.byref(nb), ctypes.byref(st), None)
    assert code == b.PR_EINVAL and b"2*rc" in b.lib.pr_last_error()
    code = b.lib.pr_react_step(10, ctypes.c_float(10.0), None, None, None, None, None, None, 4,
                               ctypes.byref(r), 1, 1, None, 4, ctypes.byref(nb), ctypes.byref(st), None)
    assert code == b.PR_ECAP
    amb = b.Rule.make(type_a=0, a_min=1, a_max=3, d_a=-1, type_t=0, t_min=3, t_max=5, d_t=1,
                      rc=1.12, exclude_bonded=1, p=0.5)
    code = b.lib.pr_react_step(10, ctypes.c_float(10.0), None, None, None, None, None, None, 4,
                               ctypes.byref(amb), 1, 1, None, 5, ctypes.byref(nb), ctypes.byref(st), None)
    assert code == b.PR_ERULE_AMBIGUOUS
    bad_p = b.Rule.make({f: getattr(r, f) for f, _ in r._fields_}, p=1.5)
    code = b.lib.pr_react_step(10, ctypes.c_float(10.0), None, None, None, None, None, None, 4,
                               ctypes.byref(bad_p), 1, 1, None, 5, ctypes.byref(nb), ctypes.byref(st), None)
    assert code == b.PR_EINVAL
    h = ctypes.c_void_p()
    assert b.lib.pr_sys_create(ctypes.byref(h), 0, ctypes.c_float(10.0), 4, ctypes.byref(r), 1, 0,
                               None) == b.PR_EINVAL


def test_footprint_and_brick_validation():
    """The footprint model runs on the host: smaller bricks mean more sweep
    workgroups and so more per-workgroup scratch; a brick edge outside 0..6
    and n above 2^30 are refused before any device call."""
    from paper_1409_7498_amd import binding as b
    from paper_1409_7498_amd import workload
    n = 50000
    d = dict(n=n, L=workload.box_for(n), B=4, rule=workload.rule_for("step", workload.RC, 0.01),
             seed=1, kind="step", gen_seed=2, sigma0=0.1, log_cap=n)
    fp = {br: b.footprint(dict(d, brick=br), 100) for br in range(7)}
    assert fp[0] == fp[4]
    assert fp[1] > fp[2] > fp[3] > fp[4] > fp[5] > fp[6]
    assert b.footprint(d, 5000) > b.footprint(d, 100)
    with pytest.raises(b.PrError) as e:
        b.footprint(dict(d, brick=7), 100)
    assert e.value.code == b.PR_EINVAL
    r = b.Rule.make(d["rule"])
    h = ctypes.c_void_p()
    assert b.lib.pr_sys_create_ex(ctypes.byref(h), n, ctypes.c_float(d["L"]), 4, ctypes.byref(r),
                                  1, 0, None, 7) == b.PR_EINVAL
    assert b.lib.pr_sys_create_ex(ctypes.byref(h), (1 << 30) + 1, ctypes.c_float(d["L"]), 4,
                                  ctypes.byref(r), 1, 0, None, 0) == b.PR_EINVAL
    best = ctypes.c_int32(0)
    bad = b.replica_desc(dict(d, brick=9))
    assert b.lib.pr_autotune(ctypes.byref(bad), 64, 0.05, 1, None, ctypes.byref(best),
                             None) == b.PR_EINVAL
    good = b.replica_desc(d)
    assert b.lib.pr_autotune(ctypes.byref(good), 64, 0.05, 0, None, ctypes.byref(best),
                             None) == b.PR_EINVAL


def test_p_from_rate():
    """p = k dt Theta (Eqs. (3)-(4)), flagged above 0.1; bad inputs refused (host only)."""
    from paper_1409_7498_amd import binding as b
    p, warn = b.p_from_rate(0.1, 0.005, 10)
    assert p == 0.1 * 0.005 * 10 and not warn
    p, warn = b.p_from_rate(2.0, 0.01, 10)
    assert abs(p - 0.2) < 1e-15 and warn
    assert b.p_from_rate(0.0, 0.005, 100) == (0.0, False)
    for bad in ((-1.0, 0.005, 10), (1.0, float("nan"), 10), (1.0, 1.0, float("inf"))):
        with pytest.raises(ValueError):
            b.p_from_rate(*bad)


def test_empty_step_without_gpu():
    """n = 0: PR_OK, no bonds, all counters zero, before any device call."""
    from paper_1409_7498_amd import binding as b
    r = b.Rule.make(type_a=1, a_min=1, a_max=4, d_a=-1, type_t=0, t_min=1, t_max=2, d_t=-1,
                    rc=1.12, exclude_bonded=1, p=0.5)
    nb = ctypes.c_int32(7)
    st = b.Stats()
    st.in_rc = 99
    code = b.lib.pr_react_step(0, ctypes.c_float(10.0), None, None, None, None, None, None, 4,
                               ctypes.byref(r), 1, 1, None, 0, ctypes.byref(nb), ctypes.byref(st),
                               None)
    assert code == b.PR_OK and nb.value == 0
    assert all(v == 0 for v in st.as_dict().values())


def test_noalloc_limit_without_gpu():
    """The allocation-free step refuses more particles than its fixed scratch
    holds, on the host, before any device call (the pointers are never read)."""
    from paper_1409_7498_amd import binding as b
    r = b.Rule.make(type_a=1, a_min=1, a_max=4, d_a=-1, type_t=0, t_min=1, t_max=2, d_t=-1,
                    rc=1.12, exclude_bonded=1, p=0.5)
    nb = ctypes.c_int32(0)
    fake = ctypes.c_void_p(0x1000)
    n = 32769
    code = b.lib.pr_react_step_noalloc(n, ctypes.c_float(40.0), fake, fake, fake, fake, fake, fake,
                                       4, ctypes.byref(r), 1, 1, fake, n // 2, ctypes.byref(nb),
                                       None, None)
    assert code == b.PR_EINVAL and b"at most 32768" in b.lib.pr_last_error()
