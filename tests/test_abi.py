"""CPU-side checks of the C-ABI library: it loads, exports every function that
include/pic.h declares, and its host-only planner validates descriptors."""
import ctypes
import os
import re

import pytest

import paper_1412_2480_amd as pic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pic.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|const char\*)\s+(pic_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = pic.lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(pic.exported_symbols())


def test_status_strings():
    L = pic.lib()
    assert L.pic_status_str(0) == b"PIC_OK"
    assert L.pic_status_str(-5) == b"PIC_E_CAPACITY"


def _run(**kw):
    base = dict(nx=64, ny=64, dx=0.1, cfl=1.0, theta=0.6, order=1,
                species=[(-1e-3, 1e-3, 16), (1e-3, 1e-3, 16)])
    base.update(kw)
    return pic.run_desc(base["nx"], base["ny"], base["dx"], base["cfl"], base["theta"],
                        base["order"], base["species"])


def test_plan_sizes_workspace():
    info = pic.plan([_run()], pic.make_options("fp64"))
    assert info.workspace_bytes > 64 * 64 * 8 * 24
    assert info.n_tiles == 16 and info.tile_slots[0] >= 16 * 256
    fast = pic.plan([_run()], pic.make_options("fp32"))
    assert fast.workspace_bytes < info.workspace_bytes


@pytest.mark.parametrize("bad", [dict(theta=0.4), dict(theta=1.2), dict(cfl=1.5),
                                 dict(order=4), dict(nx=4), dict(dx=-1.0)])
def test_plan_rejects_invalid(bad):
    with pytest.raises(pic.PicError) as ei:
        pic.plan([_run(**bad)], pic.make_options("fp64"))
    assert ei.value.code == -1


def test_plan_ragged_tiles():
    # 34 = 16 + 18 (a 2-cell tail joins the last tile), 40 = 16 + 16 + 8
    info = pic.plan([_run(nx=34, ny=40)], pic.make_options("fp64", tile=(16, 16)))
    assert info.n_tiles == 2 * 3


def test_plan_tile_shape_limits():
    # two cells per axis at least; narrow tiles are legal and no exchange
    # buffer is carved (particles go straight to their destination tile)
    for tile in ((1, 8), (8, 1)):
        with pytest.raises(pic.PicError) as ei:
            pic.plan([_run()], pic.make_options("fp64", tile=tile))
        assert ei.value.code == -1
    info = pic.plan([_run()], pic.make_options("fp32", tile=(2, 64)))
    assert info.n_tiles == 32 and info.exchange_slots == 0


def test_plan_batched_runs():
    runs = [_run(nx=128, ny=64), _run(nx=512, ny=128, order=3)]
    info = pic.plan(runs, pic.make_options("fp32"))
    assert info.n_tiles == 8 * 4 + 32 * 8
    assert info.n_cells == 128 * 64 + 512 * 128


def test_plan_learned_solver():
    base = pic.plan([_run()], pic.make_options("fp32"))
    lrn = pic.plan([_run()], pic.make_options("fp32", solver="learned", precond_slots=4))
    # network, training activations (4 x 32 channels) and 4 pairs of 6 fields
    assert lrn.workspace_bytes >= base.workspace_bytes + 64 * 64 * (4 * 32 * 4 + 4 * 6 * 8)
    # one network per distinct operator (dx, dy, cfl, theta): a second theta
    # adds a second network with its own pairs ring; a second order does not
    one = pic.plan([_run(), _run(order=3, nx=32)],
                   pic.make_options("fp32", solver="learned", precond_slots=4))
    two = pic.plan([_run(), _run(theta=0.5, nx=32)],
                   pic.make_options("fp32", solver="learned", precond_slots=4))
    assert two.workspace_bytes >= one.workspace_bytes + 32 * 64 * 4 * 6 * 8 + 9792 * 4 * 4
    o = pic.make_options("fp32", solver="learned")
    o.learned_form = 7
    with pytest.raises(pic.PicError):
        pic.plan([_run()], o)


def test_library_binds_to_torchs_hip_runtime():
    """Loading the library (as pic_plan does) before any GPU use must leave one
    HIP runtime in the process, the one torch uses: the loaded libamdhip64
    copies are counted in a fresh interpreter."""
    import subprocess
    import sys
    code = ("import paper_1412_2480_amd as pic\n"
            "pic.lib()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=root, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1", out.stdout


def test_plan_gather_option():
    """Both gathers plan the same workspace; any other value is rejected
    through the C-ABI (the binding's own check is bypassed here)."""
    a = pic.plan([_run()], pic.make_options("fp32", gather="nodal"))
    b = pic.plan([_run()], pic.make_options("fp32", gather="staggered"))
    assert a.workspace_bytes == b.workspace_bytes
    o = pic.make_options("fp32")
    o.gather = 7
    with pytest.raises(pic.PicError) as ei:
        pic.plan([_run()], o)
    assert ei.value.code == -1
    with pytest.raises(ValueError):
        pic.make_options("fp32", gather="cell")
