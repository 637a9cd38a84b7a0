"""Autotuner table: load/save/lookup on the host, and on the GPU the tuned
choice is used by AUTO closures without changing any result."""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import worklist
from workloads import configs


def _cfpq():
    import paper_1707_01007_amd as m
    from paper_1707_01007_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libcfpq.so not built")
    return m


def test_tune_table_roundtrip_on_host(tmp_path):
    cfpq = _cfpq()
    cfpq.tune_clear()
    assert cfpq.tune_get(1000) is None
    src = tmp_path / "tune.json"
    src.write_text('{"arch": "gfx950", "entries": [\n'
                   ' {"bucket": 10, "npad": 1024, "path": "bits", "tile": 32, "ms": 0.5},\n'
                   ' {"bucket": 14, "npad": 16384, "path": "mfma", "tile": 0, "ms": 2.1},\n'
                   ' {"bucket": 12, "npad": 4096, "path": "nope", "tile": 0, "ms": 1.0}\n]}\n')
    cfpq.tune_load(str(src))
    assert cfpq.tune_get(1000)["path"] == "bits" and cfpq.tune_get(1000)["tile"] == 32
    assert cfpq.tune_get(900)["npad"] == 1024          # same bucket (npad 1024)
    assert cfpq.tune_get(16000)["path"] == "mfma"
    assert cfpq.tune_get(4000) is None                   # unknown path name ignored
    out = tmp_path / "saved.json"
    cfpq.tune_save(str(out))
    cfpq.tune_clear()
    assert cfpq.tune_get(1000) is None
    cfpq.tune_load(str(out))
    assert cfpq.tune_get(1000)["tile"] == 32 and cfpq.tune_get(16384)["path"] == "mfma"
    with pytest.raises(cfpq.CfpqError):
        cfpq.tune_load(str(tmp_path / "missing.json"))
    cfpq.tune_clear()


def test_batch_route_table_on_host(tmp_path):
    """The batch tuning table: hand-set entries, validation of impossible
    routes, and a save / load round trip together with the product table."""
    cfpq = _cfpq()
    cfpq.tune_clear()
    assert cfpq.batch_tune_get(768) is None
    cfpq.batch_tune_set(256, "tiles", 128)
    cfpq.batch_tune_set(512, "resident")
    cfpq.batch_tune_set(768, "tiles", 256)
    assert cfpq.batch_tune_get(256)["route"] == "tiles" and cfpq.batch_tune_get(256)["tile"] == 128
    assert cfpq.batch_tune_get(512)["route"] == "resident" and cfpq.batch_tune_get(512)["tile"] == 0
    for bad in ((768, "resident", 0), (1024, "tiles", 64), (300, "tiles", 256), (0, "tiles", 128)):
        with pytest.raises(cfpq.CfpqError):
            cfpq.batch_tune_set(*bad)
    cfpq.batch_tune_set(768, None)  # removed
    assert cfpq.batch_tune_get(768) is None
    src = tmp_path / "tune.json"
    src.write_text('{"arch": "gfx950", "entries": [\n'
                   ' {"bucket": 10, "npad": 1024, "path": "fp4", "tile": 0, "ms": 0.01}\n], "batch": [\n'
                   ' {"batch_npad": 1024, "route": "tiles", "tile": 128, "ms": 1.5, "instances": 12},\n'
                   ' {"batch_npad": 1280, "route": "resident", "tile": 0, "ms": 1.0, "instances": 3}\n]}\n')
    cfpq.tune_load(str(src))
    e = cfpq.batch_tune_get(1024)
    assert e["route"] == "tiles" and e["tile"] == 128 and e["instances"] == 12
    assert cfpq.batch_tune_get(1280) is None            # resident above 512: not a valid route, ignored
    assert cfpq.tune_get(1000)["path"] == "fp4"
    out = tmp_path / "saved.json"
    cfpq.tune_save(str(out))
    cfpq.tune_clear()
    assert cfpq.batch_tune_get(256) is None and cfpq.batch_tune_get(1024) is None
    cfpq.tune_load(str(out))
    assert cfpq.batch_tune_get(256)["tile"] == 128 and cfpq.batch_tune_get(512)["route"] == "resident"
    assert cfpq.batch_tune_get(1024)["tile"] == 128 and cfpq.tune_get(1000)["path"] == "fp4"
    cfpq.tune_clear()


@pytest.mark.gpu
def test_autotune_choice_is_used_and_exact():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfpq = _cfpq()
    cfpq.tune_clear()
    for n in (700, 2048):
        e = cfpq.autotune(n)
        assert e["path"] in ("fp4", "mfma", "bits") and e["ms"] > 0 and len(e["candidates_ms"]) >= 2
        assert min(e["candidates_ms"].values()) == pytest.approx(e["ms"])
        inst = configs.config3(n)
        res = cfpq.closure(inst.n, inst.edges, inst.grammar)
        assert res.stats["path_used"] == {"bits": 1, "mfma": 2, "fp4": 5}[e["path"]]
        assert np.array_equal(cfpq.result_bits(res), worklist.closure(inst.n, inst.edges, inst.grammar))
    # a forced choice through the table: every variant gives the same bits
    inst = configs.config3(1024)
    want = worklist.closure(inst.n, inst.edges, inst.grammar)
    for text in ('"path": "bits", "tile": 8', '"path": "bits", "tile": 32', '"path": "mfma", "tile": 0'):
        p = os.path.join(os.environ.get("TMPDIR", "/tmp"), "cfpq_tune_test.json")
        with open(p, "w") as f:
            f.write('{"entries": [\n {"bucket": 10, "npad": 1024, ' + text + ', "ms": 1.0}\n]}\n')
        cfpq.tune_clear()
        cfpq.tune_load(p)
        res = cfpq.closure(inst.n, inst.edges, inst.grammar)
        assert np.array_equal(cfpq.result_bits(res), want), text
    cfpq.tune_clear()
