"""Host logic of the autotuner: cache keys, persistence, selection."""
import pytest

pytest.importorskip("torch")


@pytest.fixture()
def at(tmp_path, monkeypatch):
    monkeypatch.setenv("KD_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_1410_5420_amd import autotune

    return autotune


def test_defaults_without_cache(at):
    assert at.best_options("plain", 1 << 20, 3, "int32") == at.DEFAULTS


def test_key_buckets_sizes_by_log2(at):
    assert at.cache_key("plain", 1 << 20, 3, "int32") == at.cache_key("plain", (1 << 20) + 5, 3, "int32")
    assert at.cache_key("plain", 1 << 20, 3, "int32") != at.cache_key("plain", 1 << 22, 3, "int32")
    assert at.cache_key("plain", 1 << 20, 3, "int32") != at.cache_key("learned", 1 << 20, 3, "int32")


def test_select_fastest_and_persist(at):
    res = [{"config": {"cutover": 1024, "leaf_blocks": 2048}, "ms": 3.0},
           {"config": {"cutover": 2048, "leaf_blocks": 1024}, "ms": 2.5},
           {"config": {"cutover": 4096, "leaf_blocks": 1024}, "ms": 2.5}]
    best = at.select(res)
    assert best["config"] == {"cutover": 2048, "leaf_blocks": 1024}
    entries = at.load()
    entries[at.cache_key("plain", 1 << 24, 3, "int32")] = {"config": best["config"], "ms": best["ms"]}
    at.save(entries)
    assert at.best_options("plain", 1 << 24, 3, "int32") == {"cutover": 2048, "leaf_blocks": 1024}
    assert at.best_options("plain", 1 << 10, 3, "int32") == at.DEFAULTS


def test_select_needs_results(at):
    with pytest.raises(ValueError):
        at.select([])


def test_candidates_are_valid_options(at):
    for c in at.CANDIDATES:
        assert c["cutover"] in (1024, 2048, 4096)
        assert 256 <= c["leaf_blocks"] <= 16384
        assert c["records"] in (0, 1, 2)


def test_level_forms_of_the_plain_form(at):
    """The plain form tries level forms 1 and 4 at every k and deferred
    partitioning (form 3) from k = 5 on; the other forms have no level knob."""
    small = at.candidates_for("plain", 3)
    assert sorted({c["level"] for c in small}) == [1, 4]
    assert len(small) == 2 * len(at.CANDIDATES)
    big = at.candidates_for("plain", 8)
    assert sum(c["level"] == 3 for c in big) == len(at.CANDIDATES)
    assert all("level" not in c for c in at.candidates_for("batched", 8))
    assert all("level" not in c for c in at.candidates_for("learned", 8))


def test_coordinate_order_covers_every_knob(at):
    """Coordinate descent sweeps the level form (plain), the cutover, the
    finish grid, the record completion, the radix digit width and tile size,
    and (learned) the learned sorts; each knob's first value is its default."""
    plain = dict(at.coordinate_order("plain", 3))
    assert plain["digit_bits"] == (8, 11) and plain["sort_tile"] == (4096, 8192)
    assert plain["level"] == (4, 1) and plain["cutover"][0] == 1024
    assert "level" not in dict(at.coordinate_order("batched", 3))
    assert "learned_sorts" in dict(at.coordinate_order("learned", 3))
    assert 3 in dict(at.coordinate_order("plain", 6))["level"]
    for name, vals in at.coordinate_order("learned", 8):
        assert len(set(vals)) == len(vals) >= 2, name
