"""Every checked HIP call on the run path fails once, in turn, in the
fault-injection test build (libkdss_fi.so, compiled with KDSS_FAULT_INJECTION):
the entry point returns KDSS_EHIP with its message, and the plan and tree stay
usable and freeable -- a fresh upload and run afterwards equals the oracle.
The injected failure is reported after the call has run, so nothing on the
device is skipped half-way through a kernel."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import pytest

from paper_2403_05775_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def FI():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_05775_amd import kdss
    path = os.path.join(os.path.dirname(kdss.LIB_PATH), "libkdss_fi.so")
    L = kdss.lib_at(path)
    L.kdss_debug_inject_hip_failure.argtypes = [C.c_long]
    L.kdss_debug_inject_hip_failure.restype = None
    return kdss, L


def _tree(kdss, L, g, k):
    c, keep = kdss._csr(g)
    h = C.c_void_p()
    assert L.kdss_sct_build(C.byref(c), k, 0, C.byref(h)) == 0
    return h


def _plan(kdss, L, tree, T, **kw):
    o = kdss.Opts(kw.get("width", 0), 0, kw.get("every", 0), kw.get("timing", 0), 0, 0, kw.get("schedule", 0))
    p = C.c_void_p()
    assert L.kdss_plan_create(tree, T, 0, C.byref(o), C.byref(p)) == 0
    st = kdss.PlanStats()
    assert L.kdss_plan_info(p, C.byref(st)) == 0
    return p, st


def _upload_run(kdss, L, p, st, n, T):
    ws = torch.empty(st.workspace_bytes, dtype=torch.uint8, device="cuda")
    r = torch.empty(n * (2 if st.width == 128 else 1), dtype=torch.int64, device="cuda")
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    res = kdss.Result()
    rows = (kdss.TraceRow * (T + 1))()
    s = torch.cuda.current_stream().cuda_stream
    rc = L.kdss_plan_upload(p, ws.data_ptr(), ws.numel(), s)
    if rc == 0:
        rc = L.kdss_run(p, ws.data_ptr(), ws.numel(), T, None, r.data_ptr(), order.data_ptr(),
                        C.cast(rows, C.POINTER(kdss.TraceRow)), T + 1, C.byref(res), s)
    torch.cuda.synchronize()
    return rc, res, r, order


@pytest.mark.parametrize("case", ["plain", "trace", "wide", "timed"])
def test_every_hip_error_path_of_a_run(FI, oracle_mod, case):
    kdss, L = FI
    g = synth.chung_lu(1500, 12000, 2.3, seed=71, planted=15)
    k, T = 4, 3
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, k, T)
    tree = _tree(kdss, L, g, k)
    kw = dict(every=1 if case == "trace" else 0, width=128 if case == "wide" else 0,
              timing=1 if case == "timed" else 0)
    fired = 0
    for after in range(1, 400):
        p, st = _plan(kdss, L, tree, T, **kw)
        L.kdss_debug_inject_hip_failure(after)
        rc, res, r, order = _upload_run(kdss, L, p, st, g.n, T)
        L.kdss_debug_inject_hip_failure(0)
        if rc == 0:   # past the last checked call: nothing fired
            break
        assert rc == kdss.EHIP, (after, rc)
        assert b"injected failure" in L.kdss_last_error(), after
        fired += 1
        # the same plan, uploaded again, runs correctly; then it is freed
        rc, res, r, order = _upload_run(kdss, L, p, st, g.n, T)
        assert rc == 0
        got = kdss.loads_to_numpy(r, g.n, st.width)
        assert [int(x) for x in got] == [int(x) for x in ref["r"]], after
        assert (res.size, res.dens_num.value) == (ref["size"], ref["dens_num"]), after
        L.kdss_plan_free(p)
    else:
        pytest.fail("the injected failure kept firing")
    # the run that nothing interrupted is correct too
    got = kdss.loads_to_numpy(r, g.n, st.width)
    assert [int(x) for x in got] == [int(x) for x in ref["r"]]
    L.kdss_plan_free(p)
    L.kdss_sct_free(tree)
    print(f"{case}: {fired} checked HIP calls failed in turn", flush=True)
    assert fired >= 10
