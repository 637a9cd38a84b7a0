"""bench.py's command-line contract on the host: more than one GPU is refused
with a message before anything touches a device, the profiling options exist,
and the CPU baseline object carries the fields the benchmark line needs."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _bench(*args, timeout=120):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode != 0
    assert "single GPU" in r.stderr
    assert r.stdout.strip() == ""  # no benchmark line


def test_options():
    r = _bench("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--gpus", "--headline-only", "--section", "--no-cpu-baseline"):
        assert opt in r.stdout, opt


def test_cpu_baseline_fields():
    """The CPU baseline object: the oracle's single-thread time to the fixpoint
    on a sample of the workload's recipe, in the metric's unit, with the
    host's core count, the full-size oracle time, the BLAS product rate and
    the all-core bit-packed closure as separate fields.  The GPU closure (for the sample's bit-op count) is a
    stand-in here that returns the oracle's own bits."""
    import types

    import numpy as np

    import bench
    from oracle import worklist
    from workloads import configs

    class FakeGpu:
        def closure(self, n, edges, grammar, **kw):
            e = np.asarray(edges)
            return types.SimpleNamespace(stats={"bitops": 1e12}, bits=worklist.closure(n, e, grammar))

        def result_bits(self, res):
            return res.bits

    fake_torch = types.SimpleNamespace(from_numpy=lambda a: types.SimpleNamespace(cuda=lambda: a))
    inst = configs.config3(1024)
    cb = bench.cpu_baseline(FakeGpu(), fake_torch, inst, sample_n=512, closure_bitops=1e12)
    assert cb["kind"] == "oracle_closure" and cb["unit"] == "Gbitop/s" and cb["cores"] == 1
    assert cb["value"] > 0 and cb["time_to_solution_s"] > 0 and cb["identical_to_gpu"]
    assert cb["host_nproc"] >= 1 and "n=512" in cb["sample"]
    assert cb["full_size"]["time_to_solution_s"] > 0
    assert cb["blas_product"]["value"] > 0 and "n=1024" in cb["blas_product"]["sample"]
    # the all-core bit-packed closure of the whole workload, checked against the oracle's digest
    bs = cb["bitset_closure"]
    assert bs["value"] > 0 and bs["threads"] == cb["host_nproc"] and bs["n"] == 1024
    assert bs["identical_to_oracle_digest"] is True and bs["jacobi_loops"] > 1


def test_committed_traffic_matches_the_kernel_sources():
    """roofline.traffic comes from the committed rocprofv3 summaries only while
    the MFMA kernel's sources are the ones they were measured on."""
    import bench
    src = ["paper_1707_01007_amd/csrc/mfma_tile.h", "paper_1707_01007_amd/csrc/kernels_mfma.hip"]
    for md, kern in (("fp4_product_er16384_dyck.md", bench.fp4_kernel_name(bench.FP4_DEFAULT_TILE)),
                     ("mfma_product_er16384_dyck.md", "mfma_product_kernel<false, 2>")):
        t = bench.profiled_traffic(md, kern, src)
        assert t is not None, md
        assert 1.342e8 <= t < 1.342e8 * 16  # at least the algorithmic 4 x 32 MiB
