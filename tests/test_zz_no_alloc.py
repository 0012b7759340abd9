"""orca_step_noalloc (the step on the library's own scratch array, for
callers that cannot allocate) against orca_step on a caller workspace,
through the C ABI: identical results bit for bit on consecutive calls whose
crowd shrinks, and the FP64 oracle's parity contract on each."""
import ctypes

import numpy as np
import pytest

from paper_2008_11578_amd import scenarios

from parity import as_dict, compare_step

pytestmark = pytest.mark.gpu


def _run(st_np, params, noalloc):
    import torch
    from paper_2008_11578_amd import orca
    st = orca.State.from_arrays(st_np)
    n = st.n
    out = st.clone()
    status = torch.zeros(n, dtype=torch.uint8, device="cuda")
    p = orca.make_params(params)
    ain = st.agents_in()
    aout = orca.AgentsOut(orca._ptr(out.px), orca._ptr(out.py), orca._ptr(out.vx),
                          orca._ptr(out.vy), orca._ptr(status))
    stream = orca._stream_handle()
    if noalloc:
        rc = orca.lib().orca_step_noalloc(ctypes.byref(ain), ctypes.byref(aout), n,
                                          ctypes.byref(p), stream)
    else:
        ws = orca.Workspace(n)
        rc = orca.lib().orca_step(ctypes.byref(ain), ctypes.byref(aout), n, ctypes.byref(p),
                                  ws.ptr(), ws.nbytes, stream)
    assert rc == 0, orca.status_string(rc)
    torch.cuda.synchronize()
    res = {k: getattr(out, k).cpu().numpy() for k in ("px", "py", "vx", "vy")}
    res["status"] = status.cpu().numpy()
    return res


def _same(a, b):
    for k in ("px", "py", "vx", "vy", "status"):
        np.testing.assert_array_equal(a[k].view(np.uint32) if a[k].dtype == np.float32 else a[k],
                                      b[k].view(np.uint32) if b[k].dtype == np.float32 else b[k],
                                      err_msg=k)


def test_noalloc_equals_workspace_step_on_shrinking_crowds():
    from paper_2008_11578_amd import orca
    # largest accepted crowd, then the mixed crowd, then the 256-agent one:
    # each call reuses the array the previous (larger) one left behind
    big = scenarios.uniform_square(orca.NOALLOC_N_MAX, 1100.0, seed=31, n_vehicles=2000,
                                   params=scenarios.c2_mixed().params)
    for name, sc, check_oracle in (("max", big, False),
                                   ("mixed", scenarios.c2_mixed(), True),
                                   ("plain", scenarios.c1_plain(), True)):
        st = as_dict(sc)
        print("noalloc", name, sc.n, flush=True)
        a = _run(st, sc.params, noalloc=True)
        b = _run(st, sc.params, noalloc=False)
        _same(a, b)
        if check_oracle:
            compare_step(st, sc.params, gpu=a)


def test_noalloc_repeated_steps_follow_workspace_steps():
    """Five steps of the mixed crowd on the scratch array (its kept
    neighbour distances carried from step to step) equal five steps on one
    kept caller workspace."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c2_mixed()
    a = orca.State.from_arrays(sc)
    b = orca.State.from_arrays(sc)
    ws = orca.Workspace(sc.n)
    for s in range(5):
        print("noalloc step", s, flush=True)
        orca.step_noalloc(a, sc.params, out=a)
        orca.step(b, sc.params, ws, out=b)
        torch.cuda.synchronize()
        for k in ("px", "py", "vx", "vy"):
            assert torch.equal(getattr(a, k), getattr(b, k)), (s, k)
