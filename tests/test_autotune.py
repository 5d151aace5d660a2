"""The tile table's loader (host only): a table measured on other kernels is
not installed, an empty current table is reported as the default winning
everywhere, and a current table with entries is installed."""
import json

from paper_1904_11563_amd import autotune, bpx


def _write(path, entries, source):
    with open(path, "w") as f:
        json.dump({"meta": {"gemm_source": source}, "entries": entries}, f)


def test_load_labels_and_staleness(tmp_path):
    p = str(tmp_path / "tiles.json")
    assert autotune.load(p) == "none"
    _write(p, {"1188": 1}, "0" * 16)
    assert autotune.load(p) == "stale"
    _write(p, {}, autotune.kernel_source_hash())
    assert autotune.load(p) == "default won every bucket"
    _write(p, {str(autotune.index(bpx.PREC_BF16X3, 256, 1024, 1024)): 1},
           autotune.kernel_source_hash())
    try:
        assert autotune.load(p) == "autotuned (1 overrides)"
    finally:
        bpx.set_tile_table(None)


def test_default_tile_is_a_compiled_shape():
    assert 0 <= autotune.DEFAULT_TILE < bpx.tile_count(bpx.PREC_BF16X3)


def test_accept_rule():
    # a real win within the bucket's share is kept
    assert autotune.accept(4.70, 4.50, 0.10)
    # under 1 %: noise
    assert not autotune.accept(4.70, 4.66, 0.50)
    # larger than the bucket could save (1.5 x its 0.1 % share): noise
    assert not autotune.accept(4.70, 4.60, 0.001)
    # a loss is never kept
    assert not autotune.accept(4.70, 4.80, 0.50)
