"""bench.py's command-line contract that needs no GPU: one GPU only, any other count exits with
a message before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workloads_listed():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for w in ("stream", "plain", "star", "batch", "skew", "rows", "radix", "sort", "calib"):
        assert w in r.stdout
    for opt in ("--skew-budget-gib", "--skew-scramble", "--radix-budget-gib", "--sort-budget-gib"):
        assert opt in r.stdout


def test_scramble40_is_a_bijection_on_samples():
    """The skew workload's key scramble keeps keys in [0, 2^40) and never maps two keys to one (each
    step, an odd multiply or an xor-shift mod 2^40, is invertible)."""
    import numpy as np
    import datagen
    rng = np.random.default_rng(4)
    k = np.unique(np.concatenate([np.arange(1, 1 << 18), rng.integers(0, 1 << 40, 1 << 18)])).astype(np.int64)
    s = datagen.scramble40(k.copy())
    assert s.min() >= 0 and s.max() < (1 << 40)
    assert len(np.unique(s)) == len(k)
