"""Host logic of the per-size autotuner (no GPU): candidate restrictions,
objective selection (section V.A's order), and config lookup by size and
objective."""
import pytest

from paper_2211_07260_amd import autotune


def test_candidates_respect_thread_and_lds_limits():
    for f in autotune.FILTERS:
        cs = autotune.candidates(f)
        assert cs and len(set(cs)) == len(cs)
        for bx, by, tx, ty, pad, rp in cs:
            assert bx * by <= 1024 and rp == 0 and tx in (1, 2, 4, 8) and ty in (1, 2, 4, 8)
            pitch = (bx * tx + f - 1 + 3) // 4 * 4 + 4 * pad
            assert 4 * pitch * (by * ty + f - 1) <= 163840
    # a larger filter needs a larger halo: never more candidates
    assert len(autotune.candidates(17)) <= len(autotune.candidates(3))


def test_pick_orders_by_objective_then_other_then_index():
    recs = [dict(t_run_s=1.0, e_run_j=5.0), dict(t_run_s=2.0, e_run_j=3.0), dict(t_run_s=1.0, e_run_j=4.0),
            dict(t_run_s=3.0, e_run_j=3.0), dict(t_run_s=2.0, e_run_j=3.0)]
    assert autotune.pick(recs, "time") == 2      # time ties broken by energy
    assert autotune.pick(recs, "energy") == 1    # energy tie (1, 3, 4) -> lower time (1 and 4) -> earlier
    with pytest.raises(ValueError):
        autotune.pick(recs, "power")


def _store():
    e = lambda c: {"config": list(c)}
    return {"configs": {"5": {"256": {"config": [32, 8, 4, 4, 1, 0], "time": e((32, 8, 4, 4, 1, 0)),
                                      "energy": e((16, 16, 8, 4, 0, 0))},
                              "1024": {"config": [64, 4, 2, 2, 0, 0]}}}}


def test_lookup_nearest_bucket_and_objective():
    st = _store()
    assert autotune.lookup(st, 5, 300) == (32, 8, 4, 4, 1, 0)
    assert autotune.lookup(st, 5, 300, "energy") == (16, 16, 8, 4, 0, 0)
    # 512 is nearer 256 than 1024 in log-size only when below their geometric mean
    assert autotune.lookup(st, 5, 511) == (32, 8, 4, 4, 1, 0)
    assert autotune.lookup(st, 5, 513, "energy") == (64, 4, 2, 2, 0, 0)  # a time-only bucket serves both
    assert autotune.lookup(st, 9, 300) == autotune.DEFAULT
    assert autotune.lookup(None, 5, 300, "energy") == autotune.DEFAULT
    with pytest.raises(ValueError):
        autotune.lookup(st, 5, 300, "joules")


def test_stored_store_has_both_objectives_or_time_only():
    st = autotune.load()
    if st is None:
        pytest.skip("no committed store")
    for f, table in st["configs"].items():
        for side, e in table.items():
            assert len(e["config"]) == 6
            for obj in ("time", "energy"):
                if obj in e:
                    assert len(e[obj]["config"]) == 6
                    assert e[obj]["t_batch_s"] > 0
