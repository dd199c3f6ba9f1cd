"""The C-ABI library loads on the CPU, exports every symbol include/sail.h
declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sail.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sail_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def S():
    from paper_1609_07936_amd import sail
    sail.lib()
    return sail


def test_every_declared_symbol_is_exported(S):
    names = _declared()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(S.lib(), n)]
    assert not missing, missing


def test_binding_structs_match_the_header(S, tmp_path):
    """Every struct the binding passes by pointer has the size and field
    offsets the C compiler gives the header's declaration."""
    structs = {"sail_schedule": S.ScheduleC, "sail_job": S.JobC, "sail_job_result": S.JobResultC,
               "sail_server_stats": S.ServerStatsC, "sail_server_config": S.ServerConfigC,
               "sail_block_record": S.BlockRecordC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sail.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_host_only_entry_points(S):
    L = S.lib()
    sc = S.ScheduleC()
    L.sail_schedule_defaults(ctypes.byref(sc))
    # Sec. 3 defaults: blocks of 100 sweeps, a quarter branched, t = 0.1, p = 1, m = 2
    assert (sc.branch_every, sc.branch_fraction, sc.imprint_t, sc.amp_p, sc.amp_m) == (100, 0.25, 0.1, 1.0, 2)
    assert L.sail_status_string(0) == b"ok" and L.sail_status_string(2) == b"sum rules infeasible"
    fb = S.footprint_bytes(512, 128, 16384)
    # spectra [N_w][N_omega] and reconstructions [N_w][N_tau] in FP64, plus tables and per-walker scalars
    assert 16384 * (512 + 128) * 8 <= fb < 16384 * (512 + 128) * 8 * 1.2
    assert S.footprint_bytes(0, 128, 10) == 0


def test_invalid_arguments_rejected_before_device(S):
    om = (np.arange(64) + 0.5) * (10 / 64)
    tau = 0.05 * np.arange(1, 33)
    F = np.exp(-tau)
    with pytest.raises(S.SailError) as e:
        S.Problem(om[:2], tau, F, None, 1.0, 2.0)
    assert e.value.status == 1
    with pytest.raises(S.SailError) as e:
        S.Problem(om, tau, F, None, 1.0, 20.0)  # mean frequency outside the window
    assert e.value.status == 2
    with pytest.raises(S.SailError) as e:
        S.Problem(om, tau, F, -np.ones(32), 1.0, 2.0)
    assert e.value.status == 1
    bad = om.copy()
    bad[5] += 1e-3
    with pytest.raises(S.SailError) as e:
        S.Problem(bad, tau, F, None, 1.0, 2.0)
    assert e.value.status == 1
    Fn = F.copy()
    Fn[3] = np.nan
    with pytest.raises(S.SailError) as e:
        S.Problem(om, tau, Fn, None, 1.0, 2.0)
    assert e.value.status == 1


def test_too_many_bins_for_one_workgroup_is_refused(S):
    """The resync stages eight spectra per workgroup in LDS (160 KiB on
    gfx950), which bounds N_omega at 2556: a larger grid is refused with a
    message naming the LDS need, before any device is touched."""
    tau = 0.05 * np.arange(1, 33)
    F = np.exp(-tau)
    for n in (2557, 4096):
        om = (np.arange(n) + 0.5) * (10 / n)
        with pytest.raises(S.SailError) as e:
            S.Problem(om, tau, F, None, 1.0, 2.0)
        assert e.value.status == 1 and "LDS" in str(e.value), str(e.value)


def test_schedule_fields_validated_on_the_host(S):
    """The job footprint (host only) is 0 for schedules whose smoothing,
    adaptive-branching or self-cooling fields are out of range, and positive
    for the paper's protocol."""
    T = np.ones(300)
    om = (np.arange(64) + 0.5) * (10 / 64)
    tau = 0.05 * np.arange(1, 33)

    def foot(**kw):
        return S.Server.job_footprint(om, tau, 64, S.Schedule(T, **kw), S.SAIL_FP64)

    assert foot(smooth=0.01, adaptive=1, self_cool=1, boil_blocks=1, cool_blocks=1) > 0
    for bad in (dict(smooth=0.6), dict(smooth=-0.1), dict(adaptive=2), dict(self_cool=2),
                dict(self_cool=1, cool_blocks=0), dict(self_cool=1, boil_blocks=-1)):
        assert foot(**bad) == 0, bad


def test_host_side_refusals_of_the_failure_handling_entry_points(S):
    """Watchdog, per-job cancel and poll reject a NULL handle before touching
    any device."""
    L = S.lib()
    assert L.sail_set_watchdog(None, 1e-9) == 1
    a, b = ctypes.c_int(), ctypes.c_int()
    assert L.sail_watchdog_report(None, ctypes.byref(a), ctypes.byref(b)) == 1
    state = ctypes.c_int()
    assert L.sail_server_poll(None, 1, ctypes.byref(state)) == 1
    assert L.sail_server_cancel(None, 1) == 1
    assert L.sail_read_event_margins(None, 1, None, None) == 1
    assert L.sail_set_block_log(None, 4) == 1
    assert L.sail_read_block_log(None, None, 0, None, None, None) == 1


def test_no_device_reports_device_error(S):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    om = (np.arange(64) + 0.5) * (10 / 64)
    tau = 0.05 * np.arange(1, 33)
    with pytest.raises(S.SailError) as e:
        S.Problem(om, tau, np.exp(-tau), None, 1.0, 2.0)
    assert e.value.status == 4


def test_allocator_hook_takes_both_functions_or_neither(S):
    """sail_set_allocator refuses a half hook and accepts a pair or a reset;
    no device is touched."""
    L = S.lib()
    assert L.sail_set_allocator(S._ALLOC_FN(lambda n, d, u: None), S._FREE_FN(), None) == 1
    assert b"both" in L.sail_last_error()
    assert L.sail_set_allocator(S._ALLOC_FN(), S._FREE_FN(lambda p, n, d, u: None), None) == 1
    with pytest.raises(ValueError):
        S.set_allocator(lambda n, d: 0, None)
    S.set_allocator(lambda n, d: 0, lambda p, n, d: None)
    S.set_allocator(None, None)
    assert L.sail_set_allocator(S._ALLOC_FN(), S._FREE_FN(), None) == 0
