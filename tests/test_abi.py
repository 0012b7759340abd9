"""The C ABI on the CPU: liborca.so loads, exports every function that
include/orca.h declares, and rejects bad arguments on the host before any
launch (no GPU needed: none of these calls reaches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def orca_mod():
    from paper_2008_11578_amd import build, orca
    build.build(force=False)
    orca.lib()
    return orca


def declared_functions():
    text = open(os.path.join(ROOT, "include", "orca.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(orca_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(orca_mod):
    names = declared_functions()
    assert {"orca_step", "orca_build_grid", "orca_step_batched", "orca_workspace_bytes"} <= set(names)
    lib = orca_mod.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_struct_sizes_match_header(orca_mod):
    assert ctypes.sizeof(orca_mod.OrcaParams) == 4 * 4 + 4 + 4 + 16 + 4 + 8 + 8
    assert ctypes.sizeof(orca_mod.AgentsIn) == 9 * 8
    assert ctypes.sizeof(orca_mod.AgentsOut) == 5 * 8
    assert ctypes.sizeof(orca_mod.OrcaBatch) == 8 + 4 + 4 + 8 + 4 + 4 + 8 + 8 + 8


def test_status_strings(orca_mod):
    assert orca_mod.status_string(0) == "ok"
    assert "invalid" in orca_mod.status_string(-1)
    assert "workspace" in orca_mod.status_string(-2)
    assert orca_mod.status_string(12345) == "unknown status"
    assert "gfx950" in orca_mod.version()


def test_workspace_bytes_monotone(orca_mod):
    wb = orca_mod.workspace_bytes
    assert wb(-1) == 0
    prev = 0
    for n in (0, 1, 100, 10_000, 1 << 20):
        v = wb(n)
        assert v >= prev and v % 256 == 0
        prev = v
    assert wb(1000, max_cells=1 << 20) > wb(1000, max_cells=16)
    assert wb(1000, n_scenes=10) > 0


def _params(orca_mod, **kw):
    d = dict(dt=0.1, time_horizon=2.0, neighbor_dist=5.0, cell_size=0.0, max_neighbors=10,
             pref_is_goal=1, f=((0.5, 1.0), (0.0, 0.5)), par_eps=1e-5)
    d.update(kw)
    return orca_mod.make_params(d)


FAKE = 0x1000  # non-null address never dereferenced: validation fails first


def _in_fake(orca_mod):
    return orca_mod.AgentsIn(*([FAKE] * 9))


def _out_fake(orca_mod):
    return orca_mod.AgentsOut(FAKE, FAKE, FAKE, FAKE, None)


@pytest.mark.parametrize("kw,code", [
    (dict(max_neighbors=0), -4), (dict(max_neighbors=33), -4), (dict(dt=0.0), -1),
    (dict(dt=float("nan")), -1), (dict(time_horizon=-1.0), -1), (dict(neighbor_dist=0.0), -1),
    (dict(cell_size=-1.0), -1), (dict(pref_is_goal=2), -1), (dict(par_eps=-1.0), -1),
    (dict(accel=(-1.0, 0.0)), -1), (dict(accel=(0.0, float("inf"))), -1),
    (dict(accel=(0.0, float("nan"))), -1),
    (dict(turn=(-1.0, 0.0)), -1), (dict(turn=(0.0, float("inf"))), -1),
    (dict(turn=(float("nan"), 0.0)), -1),
])
def test_step_rejects_bad_params(orca_mod, kw, code):
    lib = orca_mod.lib()
    p = _params(orca_mod, **kw)
    ain, aout = _in_fake(orca_mod), _out_fake(orca_mod)
    rc = lib.orca_step(ctypes.byref(ain), ctypes.byref(aout), 100, ctypes.byref(p), FAKE,
                       1 << 30, None)
    assert rc == code


def test_step_argument_errors(orca_mod):
    lib = orca_mod.lib()
    p = _params(orca_mod)
    ain, aout = _in_fake(orca_mod), _out_fake(orca_mod)
    # n = 0 is a no-op even with null buffers
    assert lib.orca_step(None, None, 0, ctypes.byref(p), None, 0, None) == 0
    assert lib.orca_step(ctypes.byref(ain), ctypes.byref(aout), -1, ctypes.byref(p), FAKE, 1 << 30,
                         None) == -1
    assert lib.orca_step(ctypes.byref(ain), ctypes.byref(aout), 10, None, FAKE, 1 << 30, None) == -1
    # null workspace, null input arrays, null outputs
    assert lib.orca_step(ctypes.byref(ain), ctypes.byref(aout), 10, ctypes.byref(p), None, 1 << 30,
                         None) == -1
    bad_in = orca_mod.AgentsIn(*([FAKE] * 8 + [None]))
    need = orca_mod.workspace_bytes(10)
    assert lib.orca_step(ctypes.byref(bad_in), ctypes.byref(aout), 10, ctypes.byref(p), FAKE,
                         need, None) == -1
    bad_out = orca_mod.AgentsOut(FAKE, None, FAKE, FAKE, None)
    assert lib.orca_step(ctypes.byref(ain), ctypes.byref(bad_out), 10, ctypes.byref(p), FAKE,
                         need, None) == -1
    # workspace too small
    assert lib.orca_step(ctypes.byref(ain), ctypes.byref(aout), 10, ctypes.byref(p), FAKE, 64,
                         None) == -2
    # beyond the 2^28 agents the neighbour search addresses
    assert lib.orca_step(ctypes.byref(ain), ctypes.byref(aout), (1 << 28) + 1, ctypes.byref(p),
                         FAKE, 1 << 62, None) == -1
    assert lib.orca_build_grid(ctypes.byref(ain), 10, ctypes.byref(p), FAKE, 64, None, None,
                               None) == -2


def test_batched_argument_errors(orca_mod):
    lib = orca_mod.lib()
    ain, aout = _in_fake(orca_mod), _out_fake(orca_mod)
    B = orca_mod.OrcaBatch
    good = dict(scene_off=FAKE, n_scenes=2, params=FAKE, max_neighbors=16, mode=0, error_flag=None,
                has_accel=0, block=0, k_tile=0)

    def call(n=100, ws_bytes=1 << 30, **kw):
        d = dict(good)
        d.update(kw)
        b = B(**d)
        return lib.orca_step_batched(ctypes.byref(ain), ctypes.byref(aout), n, ctypes.byref(b),
                                     FAKE, ws_bytes, None)

    assert lib.orca_step_batched(None, None, 0, None, None, 0, None) == -1
    assert call(n=0) == 0
    assert call(n_scenes=0) == -1
    assert call(scene_off=None) == -1
    assert call(params=None) == -1
    assert call(max_neighbors=0) == -4
    assert call(max_neighbors=40) == -4
    assert call(mode=7) == -1
    assert call(has_accel=2) == -1
    assert call(block=96) == -1
    assert call(k_tile=8) == -4    # below max_neighbors
    assert call(k_tile=33) == -4
    assert call(ws_bytes=1024) == -2


def test_lifecycle_argument_errors(orca_mod):
    lib = orca_mod.lib()
    ain = _in_fake(orca_mod)
    buf = orca_mod.AgentsBuf(*([FAKE] * 9))
    need = lib.orca_lifecycle_workspace_bytes(100, 50)
    assert need > 0 and need % 256 == 0
    assert lib.orca_lifecycle_workspace_bytes(-1, 0) == 0
    assert lib.orca_lifecycle_workspace_bytes(100, 50) > lib.orca_lifecycle_workspace_bytes(100, 0)
    # leaving: null count, null arrays, small workspace
    assert lib.orca_remove_arrived(ctypes.byref(ain), ctypes.byref(buf), 100, None, None, FAKE,
                                   need, None) == -1
    bad_buf = orca_mod.AgentsBuf(*([FAKE] * 8 + [None]))
    assert lib.orca_remove_arrived(ctypes.byref(ain), ctypes.byref(bad_buf), 100, FAKE, None,
                                   FAKE, need, None) == -1
    assert lib.orca_remove_arrived(ctypes.byref(ain), ctypes.byref(buf), -1, FAKE, None, FAKE,
                                   need, None) == -1
    assert lib.orca_remove_arrived(ctypes.byref(ain), ctypes.byref(buf), 100, FAKE, None, FAKE,
                                   64, None) == -2

    # entering: too many candidates, capacity short, negative window, small workspace
    def spawn(n=100, cap=150, nc=50, t=1.0, ws_bytes=need, total=FAKE):
        return lib.orca_spawn(ctypes.byref(buf), n, cap, ctypes.byref(ain), nc, t, total, None,
                              FAKE, ws_bytes, None)

    assert spawn(nc=orca_mod.SPAWN_MAX + 1, cap=1 << 30) == -1
    assert spawn(cap=149) == -1
    assert spawn(t=-1.0) == -1
    assert spawn(t=float("inf")) == -1
    assert spawn(total=None) == -1
    assert spawn(ws_bytes=64) == -2


def test_overlap_argument_errors(orca_mod):
    lib = orca_mod.lib()
    ain = _in_fake(orca_mod)
    need = lib.orca_overlap_workspace_bytes(100)
    assert need > 0 and lib.orca_overlap_workspace_bytes(-1) == 0
    assert lib.orca_overlap_stats(ctypes.byref(ain), 100, 5.0, None, FAKE, need, None) == -1
    assert lib.orca_overlap_stats(ctypes.byref(ain), 100, 0.0, FAKE, FAKE, need, None) == -1
    assert lib.orca_overlap_stats(ctypes.byref(ain), -1, 5.0, FAKE, FAKE, need, None) == -1
    assert lib.orca_overlap_stats(ctypes.byref(ain), 100, 5.0, FAKE, FAKE, 64, None) == -2


def test_backward_accepts_acceleration_caps(orca_mod):
    lib = orca_mod.lib()
    ain = _in_fake(orca_mod)
    g1 = orca_mod.Cotangents(*([FAKE] * 4))
    g0 = orca_mod.CotangentsOut(*([FAKE] * 7))
    capped = _params(orca_mod, accel=(0.0, 3.0))
    bad = _params(orca_mod, accel=(0.0, -3.0))
    # a valid cap gets past the parameter checks (small workspace), a negative one does not
    assert lib.orca_step_backward(ctypes.byref(ain), 100, ctypes.byref(capped), ctypes.byref(g1),
                                  ctypes.byref(g0), FAKE, 64, None) == -2
    assert lib.orca_step_backward(ctypes.byref(ain), 100, ctypes.byref(bad), ctypes.byref(g1),
                                  ctypes.byref(g0), FAKE, 64, None) == -1


def test_backward_accepts_turn_caps(orca_mod):
    lib = orca_mod.lib()
    ain = _in_fake(orca_mod)
    g1 = orca_mod.Cotangents(*([FAKE] * 4))
    g0 = orca_mod.CotangentsOut(*([FAKE] * 7))
    turned = _params(orca_mod, turn=(0.0, 1.0))
    bad = _params(orca_mod, turn=(0.0, -1.0))
    # a valid cap gets past the parameter checks (small workspace), a negative one does not
    assert lib.orca_step_backward(ctypes.byref(ain), 100, ctypes.byref(turned), ctypes.byref(g1),
                                  ctypes.byref(g0), FAKE, 64, None) == -2
    assert lib.orca_step_backward(ctypes.byref(ain), 100, ctypes.byref(bad), ctypes.byref(g1),
                                  ctypes.byref(g0), FAKE, 64, None) == -1


def test_missing_library_fails_loudly(tmp_path):
    """With no liborca.so the binding raises instead of falling back to
    anything else (there is no CPU path)."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2008_11578_amd.orca as o\n"
        "o.LIB_PATH = %r\n"
        "o._lib = None\n"
        "try:\n"
        "    o.lib()\n"
        "except Exception as e:\n"
        "    print(type(e).__name__, e)\n"
        "    sys.exit(3)\n"
        "sys.exit(0)\n" % (ROOT, str(tmp_path / "liborca.so")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 3, (r.stdout, r.stderr)
    assert "missing" in r.stdout


def test_noalloc_argument_errors(orca_mod):
    """orca_step_noalloc validates everything before it touches a device: n
    above its scratch limit is ORCA_ETOOBIG, the rest as orca_step."""
    lib = orca_mod.lib()
    p = _params(orca_mod)
    ain, aout = _in_fake(orca_mod), _out_fake(orca_mod)
    n_max = orca_mod.NOALLOC_N_MAX
    assert lib.orca_step_noalloc(ctypes.byref(ain), ctypes.byref(aout), n_max + 1,
                                 ctypes.byref(p), None) == -5
    assert lib.orca_step_noalloc(ctypes.byref(ain), ctypes.byref(aout), 1 << 28,
                                 ctypes.byref(p), None) == -5
    assert lib.orca_step_noalloc(None, None, 0, ctypes.byref(p), None) == 0
    assert lib.orca_step_noalloc(ctypes.byref(ain), ctypes.byref(aout), -1, ctypes.byref(p),
                                 None) == -1
    assert lib.orca_step_noalloc(ctypes.byref(ain), ctypes.byref(aout), 10, None, None) == -1
    bad = _params(orca_mod, max_neighbors=33)
    assert lib.orca_step_noalloc(ctypes.byref(ain), ctypes.byref(aout), 10, ctypes.byref(bad),
                                 None) == -4
    bad_in = orca_mod.AgentsIn(*([FAKE] * 8 + [None]))
    assert lib.orca_step_noalloc(ctypes.byref(bad_in), ctypes.byref(aout), 10, ctypes.byref(p),
                                 None) == -1
    bad_out = orca_mod.AgentsOut(FAKE, None, FAKE, FAKE, None)
    assert lib.orca_step_noalloc(ctypes.byref(ain), ctypes.byref(bad_out), 10, ctypes.byref(p),
                                 None) == -1
    assert "no-allocation" in orca_mod.status_string(-5)
    # the largest accepted crowd fits the scratch array
    assert orca_mod.workspace_bytes(n_max) <= 16 << 20
