"""Host logic of bench.py (CPU): the algorithmic byte model of the pruned
schedule, the kernel names the counter lookup uses, the hash gate of the
committed rocprofv3 summaries, and the one-GPU refusal."""
import os
import subprocess
import sys


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_byte_model_counts_the_pruned_fields():
    n, s = 128, 8
    K = (n - 1) // 3
    KP, M = K + 1, 2 * K + 1
    Q = M * KP
    b = bench.pass_bytes(n, s, split_z=False)
    # x-pass: six y-partial fields in, three fields out, plus 39 FP64 sums per workgroup
    assert b["x_pass"] == 9 * n * n * KP * s + (n * n // 8) * 39 * 8 == 51363840
    assert b["y_inverse"] == (6 * n * Q + 6 * n * n * KP) * s
    # fused z-pass: 3 forward fields, state in/out and history in/out, 6 inverse fields
    assert b["z_pass"] == (3 * n * Q + 12 * M * Q + 6 * n * Q) * s
    assert bench.step_bytes(n, s) == b["y_inverse"] + b["x_pass"] + b["y_forward"] + b["z_pass"]


def test_byte_model_of_a_box():
    assert bench.pass_bytes(128, 8, False, nx=128) == bench.pass_bytes(128, 8, False)
    b = bench.pass_bytes(128, 8, False, nx=192)
    KP = (192 - 1) // 3 + 1
    assert b["x_pass"] == 9 * 128 * 128 * KP * 8 + (128 * 128 // 4) * 39 * 8 == 76775424


def test_kernel_names_and_counter_gate():
    sched = {"y_inverse": 1, "x_pass": 0, "y_forward": 1, "z_pass": 2, "split_z": 0}
    assert bench.kernel_of_pass("x_pass", 128, "float", sched, 1, False) == "k_xpass<float, 128, 128, 1, 0, false>"
    assert bench.kernel_of_pass("z_pass", 128, "float", sched, 1, False, nx=192) == \
        "k_zpass<float, 192, 128, 1, 2, false>"
    # the y-inverse launch that also evaluates moving kinematics is its own instantiation
    assert bench.kernel_of_pass("y_inverse", 128, "float", sched, 3, True) == "k_ypass<float, 128, 128, 1, 2, 1>"
    assert bench.kernel_of_pass("y_inverse", 128, "float", sched, 1, False) == "k_ypass<float, 128, 128, 1, 0, 1>"
    assert bench.moving_body({"wings": True}) and bench.moving_body({"free_flight": True})
    assert not bench.moving_body({"body": "sphere"}) and not bench.moving_body(None)
    assert bench.counter_traffic("no_such_workload", "k_xpass") is None
    path = os.path.join(ROOT, "profiles", "sphere128.md")
    if f"csrc_sha256: {bench.source_hash()}" in open(path).read():
        t = bench.counter_traffic("sphere128", "k_xpass<float, 128, 128, 1, 0, false>")
        assert isinstance(t, int) and t > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
