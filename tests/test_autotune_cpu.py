"""Host logic of the tile autotuner: the candidate tiles of a grid size and
the JSON cache round trip (no GPU)."""
import math

from paper_2402_06927_amd import autotune as A


def test_candidates_are_compiled_tiles_within_limits():
    for nx in (64, 100, 256, 600, 1000, 2048, 4096, 5000, 8192):
        c = A.candidates(nx)
        assert c, nx
        for nt in c:
            assert nx >= nt and math.ceil(nx / nt) <= 16
            assert (nt, A.slots(nx, nt)) in A.TILES
    assert A.candidates(4096) == [256, 512]
    assert A.candidates(64) == [64]
    assert 64 not in A.candidates(2048)  # 32 nodes per thread


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "tiles.json")
    assert A.load_cache(p) == {}
    A.save_cache(p, {4096: 256, 512: 64})
    assert A.load_cache(p) == {4096: 256, 512: 64}
