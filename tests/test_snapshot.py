"""Cycle-boundary snapshots of the twin-experiment driver (host side): the
arrays come back exactly, the file holds plain arrays only (it loads with
pickling disabled), and a snapshot of another workload, filter or seed, or of
another format version, is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2402_06927_amd import experiments as E
from paper_2402_06927_amd import workloads as W


def _state(seed=0):
    g = np.random.default_rng(seed)
    return {"m": torch.tensor(g.standard_normal((6, 100))),
            "u": torch.tensor(g.standard_normal((6, 100))),
            "m_truth": torch.tensor(g.standard_normal((1, 100))),
            "u_truth": torch.tensor(g.standard_normal((1, 100))),
            "logw": torch.tensor(g.standard_normal(6)),
            "init_stats": torch.tensor([0.5, -0.1, 0.9], dtype=torch.float64)}


def test_round_trip_is_exact(tmp_path):
    wl = W.PAPER_SHAPE.scaled(n_particles=6)
    st = _state()
    path = str(tmp_path / "s.npz")
    E.save_snapshot(path, wl, "bootstrap", 41, st)
    cyc, arrays = E.load_snapshot(path, wl, "bootstrap")
    assert cyc == 41
    assert set(arrays) == set(st)
    for k, v in st.items():
        assert arrays[k].dtype == np.float64
        np.testing.assert_array_equal(arrays[k], v.numpy())
    # plain arrays: numpy's own loader without pickling reads every entry
    with np.load(path, allow_pickle=False) as z:
        for k in z.files:
            z[k]


def test_snapshot_of_another_run_is_refused(tmp_path):
    wl = W.PAPER_SHAPE.scaled(n_particles=6)
    path = str(tmp_path / "s.npz")
    E.save_snapshot(path, wl, "tempered", 3, _state())
    with pytest.raises(ValueError, match="snapshot of"):
        E.load_snapshot(path, wl, "bootstrap")
    with pytest.raises(ValueError, match="snapshot of"):
        E.load_snapshot(path, W.PAPER_HALF.scaled(n_particles=6), "tempered")
    with pytest.raises(ValueError, match="snapshot of"):
        E.load_snapshot(path, wl.scaled(seed=wl.seed + 7), "tempered")
    bad = str(tmp_path / "v.npz")
    np.savez(bad, version=np.array(E.SNAPSHOT_VERSION + 1), workload=np.array(wl.name),
             filter=np.array("tempered"), seed=np.array(wl.seed), cycle=np.array(0))
    with pytest.raises(ValueError, match="version"):
        E.load_snapshot(bad, wl, "tempered")
