"""The ensemble autotune cache (host only): the key separates precision,
depth, size class and member count; entries survive a round trip through the
JSON file and a store keeps the other entries."""
from paper_2309_06662_amd import inputs, ocn


def test_tuning_key_separates_what_changes_the_choice():
    base = inputs.BETA_BASIN_64
    ws = [base.replace(nx=128, ny=128, nz=32), base.replace(nx=256, ny=128, nz=48)]
    k = ocn.tuning_key("fp32", ws)
    assert k == ocn.tuning_key("fp32", list(ws))
    assert k != ocn.tuning_key("fp64", ws)
    assert k != ocn.tuning_key("fp32", [ws[0], ws[1].replace(nz=64)])
    assert k != ocn.tuning_key("fp32", ws + ws)  # more members, twice the cells
    # the same size class: a few percent more cells
    assert k == ocn.tuning_key("fp32", [ws[0], ws[1].replace(nx=260)])


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "autotune.json")
    assert ocn.autotune_cache_load(path) == {}
    a = {"tend_rows": 8, "baro_fuse": 7, "persistent": 1, "ms_per_step": 12.5}
    b = {"tend_rows": 4, "baro_fuse": 6, "persistent": 0, "ms_per_step": 3.0}
    ocn.autotune_cache_store(path, "k1", a)
    ocn.autotune_cache_store(path, "k2", b)
    got = ocn.autotune_cache_load(path)
    assert got == {"k1": a, "k2": b}
    ocn.autotune_cache_store(path, "k1", b)
    assert ocn.autotune_cache_load(path) == {"k1": b, "k2": b}


def test_unreadable_cache_reads_as_empty(tmp_path):
    path = tmp_path / "autotune.json"
    path.write_text('{"fp32|nz=32": {"tend_rows": 8,')   # cut off mid-write
    assert ocn.autotune_cache_load(str(path)) == {}
    ocn.autotune_cache_store(str(path), "k", {"tend_rows": 4, "baro_fuse": 6, "persistent": 0})
    assert ocn.autotune_cache_load(str(path)) == {"k": {"tend_rows": 4, "baro_fuse": 6, "persistent": 0}}
    path.write_text("[1, 2]")                                  # valid JSON, not an object
    assert ocn.autotune_cache_load(str(path)) == {}
