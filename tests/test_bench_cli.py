"""bench.py's command-line contract and host logic that need no GPU: one GPU only, any other
count exits with a message before any device work; the default line's blocks; the batch's
sampled closed-form check."""
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
    for opt in ("--skew-budget-gib", "--skew-scramble", "--radix-budget-gib", "--sort-budget-gib", "--no-skew",
                "--no-plain", "--no-star", "--no-batch", "--batch-steps"):
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


def test_sub_block_keeps_the_workload_fields():
    """A block of the default line runs its workload with its own steps and warmup, and drops only
    the fields the headline line carries."""
    import argparse
    import bench
    seen = {}

    def run(a):
        seen["steps"], seen["warmup"] = a.steps, a.warmup
        return {"metric": "m", "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "data": "synthetic", "value": 3.0, "roofline": {"bound": "hbm"}, "cpu_baseline": {"value": 1.0}}

    args = argparse.Namespace(steps=5, warmup=1, gpus=1)
    out = bench._sub_block(run, args, 50, 10)
    assert seen == {"steps": 50, "warmup": 10}
    assert out == {"value": 3.0, "roofline": {"bound": "hbm"}, "cpu_baseline": {"value": 1.0}}
    assert args.steps == 5 and args.warmup == 1


def test_batch_checks_reject_a_wrong_job():
    """The bench's sampled closed-form check of the batched joins stops on a job whose result is
    wrong (here every result is zero, and every sampled job has matches)."""
    import pytest
    import bench
    import datagen
    b, p = datagen.batch_sizes(256)
    with pytest.raises(SystemExit, match="closed form"):
        bench._batch_checks(b, p, [[0, 0]] * 256)
