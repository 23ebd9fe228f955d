"""Host-side logic of bench.py (no GPU): the algorithmic byte counts against the arrays the binding
actually allocates, the attribution of every byte to exactly one kernel, the measured-traffic
lookup, the one-GPU guard and the single-thread oracle sample."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
from paper_1711_00289_amd import binding
from paper_1711_00289_amd import soundings as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("L", [2, 30, 46, 72])
def test_bytes_per_column_match_the_allocated_arrays(L):
    """Every input and output array the library reads or writes, counted per column: the inputs
    from the generated state's arrays that conv_state_t points at, the outputs from the binding's
    allocations (host tensors of the device path's shapes)."""
    import torch

    ld = 7
    st = S.make_state(ld, L, seed=5)
    ptrs = [f for f, t in binding.State._fields_ if t is binding.C.c_void_p]
    assert len(ptrs) == 8
    inputs = sum(np.asarray(st[f], dtype=np.float64).nbytes for f in ptrs) / ld
    per_col = lambda d: sum(v.numel() * v.element_size() for v in d.values()) / ld
    deep = per_col(binding.alloc_deep(torch, "cpu", L, ld))
    shallow = per_col(binding.alloc_shallow(torch, "cpu", L, ld))
    b = bench.bytes_per_column(L)
    assert b["inputs"] == inputs
    assert b["deep_scalars"] + b["deep_arrays"] == deep
    assert b["shallow"] == shallow
    assert b["total"] == inputs + deep + shallow
    if L == 30:
        assert b["total"] == 2996


def test_kernel_bytes_charge_every_byte_once():
    rng = np.random.default_rng(3)
    n, L = 5000, 30
    trig = (rng.random(n) < 0.15).astype(np.int32)
    sst = rng.integers(0, 7, n).astype(np.int32)
    kb = bench.kernel_bytes(L, n, trig, sst)
    assert sum(kb.values()) == n * bench.bytes_per_column(L)["total"]
    # nothing convecting: the trigger writes everything
    kb0 = bench.kernel_bytes(L, n, np.zeros(n, np.int32), np.ones(n, np.int32))
    assert kb0["trigger"] == n * bench.bytes_per_column(L)["total"]
    assert kb0["deep_plume"] == kb0["shallow_retrigger"] == kb0["shallow_plume"] == 0


def test_measured_traffic_lookup(monkeypatch):
    got = bench.measured_traffic("k_trigger")
    fetch, write = bench.MEASURED_TRAFFIC["k_trigger"]
    if got is not None:  # the kernel sources are the ones the counters were taken on
        assert got == int((2.0 * fetch + 1.0 * write) * 1024)
    assert bench.measured_traffic("k_no_such_kernel") is None
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "sources_sha256", "0" * 64)
    assert bench.measured_traffic("k_trigger") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_single_thread_oracle_sample():
    st = S.make_state(96, 30, seed=7, warm=np.ones(96, bool))
    rate, secs, n = bench.cpu_one_thread(st, stride=4)
    assert n == 24 and secs > 0 and rate == pytest.approx(n / secs)


def test_adjoint_bytes():
    """Quiet columns: status read, two gradient arrays written; an active column adds the deep
    scheme's inputs (the step's inputs less pblh and tke), two level indices and two cotangent
    arrays."""
    L, n = 30, 1000
    quiet = bench.adjoint_bytes(L, n, 0)
    assert quiet == n * (4 + 2 * L * 8)
    extra = (bench.adjoint_bytes(L, n, n) - quiet) / n
    assert extra == bench.bytes_per_column(L)["inputs"] - 2 * 8 + 2 * 4 + 2 * L * 8


def test_oracle_operation_count_and_cpu_sweep_helpers():
    """The algorithmic operation count is per column, positive, and larger for convecting columns
    (they run the plume passes); the chunk sweep's baseline runs at every chunk size; the CPU model
    is read from lscpu when it exists."""
    import oracle

    st = S.make_state(64, 30, seed=7, warm=np.ones(64, bool))
    ops = oracle.step_ops(st)
    od, osh = oracle.step(st)
    assert ops.shape == (64,) and (ops > 30 * 6).all()
    act = od["status"] == 0
    assert act.any() and (~act).any()
    assert ops[act].mean() > 1.5 * ops[~act].mean()
    mean, n = bench.oracle_ops(st, stride=4)
    assert n == 16 and mean == pytest.approx(ops[::4].mean())
    for c in bench.OMP_CHUNKS:
        rate, secs, steps = bench.cpu_baseline(st, 2, chunk=c, min_cpu_s=0.0, max_steps=1)
        assert steps == 1 and rate > 0
    m = bench.cpu_model()
    assert m is None or isinstance(m, str)
