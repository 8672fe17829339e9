"""bench.py contract checks that need no GPU: more than one GPU is refused with a message."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_a_distributed_launch_is_refused():
    r = _run([], {"WORLD_SIZE": "2"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_advection_options_are_checked():
    for args in (["--advection"], ["--workload", "porous_2d", "--advection", "--precision", "bf16"],
                 ["--workload", "porous_3d", "--advection", "--shift", "node"]):
        r = _run(args)
        assert r.returncode == 2 and "--advection" in r.stderr, (args, r.stderr)


def test_advective_step_bytes():
    """Species (2 Q) and velocity-model (Q) entries read and written once, plus the node velocity
    of the previous step read and of this one written (3 doubles each)."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.adv_bytes_per_node("D2Q9", "fp32") == 2 * 3 * 9 * 4 + 2 * 3 * 8 == 264
    assert bench.adv_bytes_per_node("D3Q19", "fp32") == 504
    assert bench.adv_bytes_per_node("D3Q19", "fp64") == 2 * 3 * 19 * 8 + 48
    assert bench.adv_bytes_per_node("D2Q5", "fp64") == 2 * 3 * 5 * 8 + 48
