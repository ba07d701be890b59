"""bench.py's command line (host only): the benchmarked block's solver form
is the default, the other workloads keep the form they were measured with,
and more than one GPU is refused with a message."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _parse(*argv):
    sys.path.insert(0, ROOT)
    import bench
    old = sys.argv
    sys.argv = ["bench.py", *argv]
    try:
        return bench.parse()
    finally:
        sys.argv = old


def test_block_form_is_the_default():
    a = _parse()
    assert (a.workload, a.scene, a.grid, a.steps, a.warmup) == ("block32", "block", 32, 8, 2)
    assert (a.precision, a.pc) == ("mixed", "additive")
    assert (a.handles, a.rigid, a.jump, a.smoother) == (144, 1e3, 0.25, 1)
    assert (a.eta_min, a.eta_max, a.endgame_ratio, a.endgame_fp64, a.coarse_move) == (3e-2, 0.1, 1e-1, 0, 0.8)


@pytest.mark.parametrize("argv", [("--workload", "batch64"), ("--scene", "gyroid", "--grid", "64"),
                                  ("--scene", "sliding")])
def test_other_workloads_keep_their_form(argv):
    a = _parse(*argv)
    assert (a.handles, a.smoother, a.endgame_fp64, a.coarse_move) == (192, 0, 1, 0.2)
    assert (a.eta_min, a.endgame_ratio) == (1e-4, 1e-3)


def test_explicit_flags_win():
    a = _parse("--handles", "176", "--smoother", "0", "--eta-min", "1e-3", "--coarse-move", "0.2")
    assert (a.handles, a.smoother, a.eta_min, a.coarse_move) == (176, 0, 1e-3, 0.2)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)
