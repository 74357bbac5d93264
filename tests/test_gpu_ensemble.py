"""Batched ensembles: members of different sizes stepped by one launch per
stage (graph-replayed after the first step) must equal the same basins stepped
alone, bitwise, at every step; tile settings and the autotuner must not change
results; a member still matches the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2309_06662_amd import inputs
from tests.helpers import masks, rel_l2

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "T", "eta", "U", "V", "eta_mean", "U_mean", "V_mean")


def _members():
    base = inputs.BETA_BASIN_64
    return [base.replace(name="m0_48x40x6", nx=48, ny=40, nz=6, depth=1500.0, tau0=0.12, seed=3),
            base.replace(name="m1_70x33x8", nx=70, ny=33, nz=8, depth=2000.0, tau0=0.07, strat_scale=700.0, seed=4),
            base.replace(name="m2_130x21x5", nx=130, ny=21, nz=5, depth=1000.0, tau0=0.18, seed=5)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_members_equal_solo_runs_at_every_replay(precision):
    from paper_2309_06662_amd import ocn

    ws = _members()
    inps = [inputs.make_inputs(w) for w in ws]
    print(f"ensemble of {len(ws)} {precision}", flush=True)
    ens = ocn.Ensemble(ws, precision, inps)
    solo = [ocn.Model(w, precision, inp) for w, inp in zip(ws, inps)]
    for step in range(4):
        ens.step(1)
        for s in solo:
            s.step(1)
        for m, (mem, s) in enumerate(zip(ens.members, solo)):
            for n in FIELDS:
                assert np.array_equal(mem.get(n), s.get(n)), (step, m, n)
    assert ens.members[1].diagnostics()["step"] == 4


def test_tile_settings_do_not_change_results():
    from paper_2309_06662_amd import ocn

    ws = _members()
    inps = [inputs.make_inputs(w) for w in ws]
    a = ocn.Ensemble(ws, "fp32", inps)
    b = ocn.Ensemble(ws, "fp32", inps)
    a.set_tiles(4, 3)
    b.set_tiles(8, 6)
    a.step(5)
    b.step(5)
    for ma, mb in zip(a.members, b.members):
        for n in FIELDS:
            assert np.array_equal(ma.get(n), mb.get(n)), n


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_persistent_queues_equal_one_workgroup_per_tile(precision):
    """Persistent workgroups over per-XCD atomic queues give bitwise the
    results of one workgroup per tile (and of the members alone), graph
    replay after graph replay."""
    from paper_2309_06662_amd import ocn

    ws = _members()
    inps = [inputs.make_inputs(w) for w in ws]
    a = ocn.Ensemble(ws, precision, inps)
    b = ocn.Ensemble(ws, precision, inps)
    a.set_tiles(0, 0, persistent=1)
    b.set_tiles(0, 0, persistent=0)
    solo = [ocn.Model(w, precision, inp) for w, inp in zip(ws, inps)]
    for step in range(4):
        a.step(1)
        b.step(1)
        for s in solo:
            s.step(1)
        for m, (ma, mb, s) in enumerate(zip(a.members, b.members, solo)):
            for n in FIELDS:
                x = ma.get(n)
                assert np.array_equal(x, mb.get(n)), (step, m, n)
                assert np.array_equal(x, s.get(n)), (step, m, n)
    # another substep grouping under the queues (an odd number of barotropic launches)
    a.set_tiles(4, 5, persistent=1)
    b.set_tiles(4, 5, persistent=0)
    a.step(3)
    b.step(3)
    for ma, mb in zip(a.members, b.members):
        for n in FIELDS:
            assert np.array_equal(ma.get(n), mb.get(n)), n


def test_autotune_cache_is_used_and_keeps_results(tmp_path):
    from paper_2309_06662_amd import ocn

    ws = _members()
    cache = str(tmp_path / "autotune.json")
    a = ocn.Ensemble(ws, "fp32")
    first = a.autotune(trial_steps=1, cache=cache)
    assert first["cached"] is False
    b = ocn.Ensemble(ws, "fp32")
    second = b.autotune(trial_steps=1, cache=cache)
    assert second["cached"] is True
    for k in ("tend_rows", "baro_fuse", "persistent"):
        assert second[k] == first[k], k
    c = ocn.Ensemble(ws, "fp32")  # default tiles
    b.step(3)
    c.step(3)
    for mb, mc in zip(b.members, c.members):
        for n in FIELDS:
            assert np.array_equal(mb.get(n), mc.get(n)), n


def test_autotune_restores_state_and_picks_a_valid_choice():
    from paper_2309_06662_amd import ocn

    ws = _members()
    ens = ocn.Ensemble(ws, "fp32")
    ens.step(2)
    before = [m.get("u") for m in ens.members]
    choice = ens.autotune(trial_steps=2)
    assert choice["tend_rows"] in (4, 8) and choice["baro_fuse"] in (5, 6, 7, 8) and choice["ms_per_step"] > 0
    assert choice["persistent"] in (0, 1) and choice["cached"] is False
    after = [m.get("u") for m in ens.members]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert ens.members[0].diagnostics()["step"] == 2
    ens.step(2)  # keeps stepping from the restored state
    assert ens.members[0].diagnostics()["nonfinite"] == 0


def test_member_matches_oracle_fp64():
    from paper_2309_06662_amd import ocn

    ws = _members()
    inps = [inputs.make_inputs(w) for w in ws]
    ens = ocn.Ensemble(ws, "fp64", inps)
    ens.step(6)
    w, inp = ws[1], inps[1]
    ref = oracle.OracleModel.from_inputs(w, inp)
    ref.step(6)
    wet, mu, mv = masks(w, inp["kbottom"])
    mk = {"u": mu, "v": mv, "T": wet}
    for n in ("u", "v", "T", "eta", "U", "V"):
        assert rel_l2(ens.members[1].get(n), ref.get(n), mk.get(n)) <= 1e-11, n
