"""The paper-style command-line driver: argument handling on the CPU (the
product itself needs the GPU and is covered by the gpu tests)."""
import numpy as np
import pytest

from paper_2408_15384_amd import cli
from paper_2408_15384_amd import inputs as I


def test_sizes_are_m_k_n():
    a = cli.parse(["300", "200", "100"])
    assert (a.M, a.K, a.N) == (300, 200, 100)
    assert a.method == "f64" and a.inputs == "uniform" and a.reps == 15 and a.warmup == 3
    A, B = cli.host_operands(a)
    assert A.shape == (300, 200) and B.shape == (200, 100) and A.dtype == np.float64


@pytest.mark.parametrize("argv", [
    ["-1", "2", "3"],                                    # negative size
    ["4", "4", "4", "--reps", "0"],                      # no timed run
    ["4", "4", "4", "--method", "f64", "--inputs", "m2e"],   # m2e is an FP32 set
    ["4", "4", "4", "--method", "strassen", "--trans-a"],
    ["3", "4", "4", "--method", "strassen"],             # odd size
    ["4", "4"],                                          # missing size
])
def test_bad_arguments_exit(argv):
    with pytest.raises(SystemExit):
        cli.parse(argv)


def test_inputs_follow_the_seeded_generators():
    a = cli.parse(["16", "8", "12", "--method", "split6", "--inputs", "normal", "--seed", "4"])
    A, B = cli.host_operands(a)
    RA, RB = I.pair("normal_f64", 16, 12, 8, seed=4)
    assert A.dtype == np.float32 and np.array_equal(A, RA.astype(np.float32)) and np.array_equal(B, RB.astype(np.float32))
    a = cli.parse(["16", "8", "12", "--method", "f32", "--inputs", "int"])
    A, _ = cli.host_operands(a)
    assert A.dtype == np.float32 and np.all(A == np.round(A)) and np.abs(A).max() <= 8


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: asking for more exits with a message before touching a device
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2", "--steps", "1", "--warmup", "0"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
