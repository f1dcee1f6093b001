"""Host logic of the batch tile tuner (no GPU): the candidate list and the
choice among timed candidates, with the GPU timing replaced by fixed numbers."""
from paper_1603_08221_amd import autotune, lbsep


def _params(dtype="f64"):
    # one member below 2^14 nodes and one above, so the size thresholds differ
    return [lbsep.make_params(80, 16, 4, 40, 0.3, 0.3, 3.0, 0.05, 0.87, dtype=dtype),
            lbsep.make_params(640, 32, 4, 40, 0.3, 0.3, 3.0, 0.05, 0.87, dtype=dtype)]


def test_candidates_cover_modes_and_rows():
    c = autotune.candidates(_params())
    assert c["node,rows2"] == {"modes": [autotune.NODE] * 2, "rows": [2, 2]}
    assert c["split,rows4"] == {"modes": [autotune.SPLIT] * 2, "rows": [4, 4]}
    assert c["split<=16384"] == {"modes": [autotune.SPLIT, autotune.NODE], "rows": [0, 0]}
    # each mode assignment comes with rows by size, 2 and 4
    assert len(c) % 3 == 0 and all(n + ",rows2" in c and n + ",rows4" in c for n in c if "rows" not in n)


def test_fp32_candidates_have_no_four_row_tiles():
    c = autotune.candidates(_params("f32"))
    assert c["node,rows2"] == {"modes": [autotune.NODE] * 2, "rows": [2, 2]}
    assert not any(n.endswith(",rows4") for n in c)
    assert len(c) % 2 == 0 and all(n + ",rows2" in c for n in c if "rows" not in n)
    # a batch with any member in another dtype keeps them
    mixed = _params("f32")[:1] + _params("f16")[1:]
    assert "node,rows4" in autotune.candidates(mixed)


def _tune(monkeypatch, ms, dtype="f64"):
    monkeypatch.setattr(autotune, "_key", lambda ps, dev: "k")
    monkeypatch.setattr(autotune, "_time_batch", lambda ps, modes, rows, *a: ms(modes, rows))
    return autotune.tune(_params(dtype))


def test_clear_winner_is_chosen(monkeypatch):
    got = _tune(monkeypatch, lambda m, r: 0.10 if (m == [autotune.NODE] * 2 and r == [4, 4]) else 0.20)
    assert got["name"] == "node,rows4" and got["rows"] == [4, 4] and got["ms_per_step"] == 0.10


def test_near_tie_goes_to_the_first_candidate(monkeypatch):
    # split<=16384,rows2 is 0.5% faster than node,rows2, which comes first
    def ms(m, r):
        if r == [2, 2] and m == [autotune.SPLIT, autotune.NODE]:
            return 0.2054
        return 0.2065 if (r == [2, 2] and m == [autotune.NODE] * 2) else 0.25
    got = _tune(monkeypatch, ms)
    assert got["name"] == "node,rows2"
    assert list(autotune.candidates(_params())).index("node,rows2") < \
        list(autotune.candidates(_params())).index("split<=16384,rows2")
    # beyond the tie margin the faster one wins
    got = _tune(monkeypatch, lambda m, r: 0.200 if (r == [2, 2] and m == [autotune.SPLIT, autotune.NODE])
                else 0.210 if (r == [2, 2] and m == [autotune.NODE] * 2) else 0.25)
    assert got["name"] == "split<=16384,rows2"


def test_each_candidate_keeps_its_best_round(monkeypatch):
    # the first round runs while the clocks rise: "node" is slow there and the
    # fastest in the second round, where the others keep their first times
    calls = []

    def ms(m, r):
        calls.append((tuple(m), tuple(r)))
        first = calls.count((tuple(m), tuple(r))) == 1
        if m == [autotune.NODE] * 2 and r == [0, 0]:
            return 0.30 if first else 0.10
        return 0.20 if first else 0.25
    got = _tune(monkeypatch, ms)
    n = len(autotune.candidates(_params()))
    assert len(calls) == 2 * n  # two rounds over every candidate
    assert got["name"] == "node" and got["ms_per_step"] == 0.10
    assert all(v == 0.20 for k, v in got["timings"].items() if k != "node")
