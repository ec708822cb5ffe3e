"""Resuming the twin-experiment driver from a cycle-boundary snapshot: four
assimilation steps in one run, and two steps, a snapshot, and a second run
that resumes from it, give bit-identical ensembles, truths and statistics
(every random draw is keyed by seed and cycle), for the three filters; the
per-step JSON log has one record per step with the run's statistics."""
import json
import sys

import numpy as np
import pytest

from paper_2402_06927_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_06927_amd import experiments as X
    from paper_2402_06927_amd import sch

    sch.lib()
    return X


@pytest.mark.parametrize("filt", ["bootstrap", "tempered", "nudged"])
def test_resume_reproduces_the_uninterrupted_run(E, filt, tmp_path):
    print("resume", filt, file=sys.stderr, flush=True)
    wl = W.PAPER_SHAPE.scaled(n_particles=12 if filt == "nudged" else 24)
    whole = E.run_twin(wl, filt, 4, jsonl=str(tmp_path / "whole.jsonl"))
    snap = str(tmp_path / "s.npz")
    first = E.run_twin(wl, filt, 2, snapshot=snap)
    rest = E.run_twin(wl, filt, 4, resume=snap, jsonl=str(tmp_path / "rest.jsonl"))
    assert rest["first_step"] == 2 and rest["n_da"] == 2
    np.testing.assert_array_equal(rest["u"], whole["u"])
    np.testing.assert_array_equal(rest["u_truth"], whole["u_truth"])
    np.testing.assert_array_equal(rest["init"], whole["init"])
    for key in ("emre", "rb", "res", "ess"):
        np.testing.assert_array_equal(np.concatenate([first[key], rest[key]]), whole[key])
    recs = [json.loads(l) for l in open(tmp_path / "whole.jsonl")]
    assert [r["step"] for r in recs] == [0, 1, 2, 3]
    for c, r in enumerate(recs):
        assert r["emre"] == whole["emre"][c] and r["ess"] == whole["ess"][c]
        if filt == "bootstrap":
            assert r["resampled"] == whole["resampled"][c]
        else:
            assert r["n_temper"] == whole["n_temper"][c]
    assert [json.loads(l)["step"] for l in open(tmp_path / "rest.jsonl")] == [2, 3]


def test_resume_past_the_end_is_refused(E, tmp_path):
    wl = W.PAPER_SHAPE.scaled(n_particles=8)
    snap = str(tmp_path / "s.npz")
    E.run_twin(wl, "bootstrap", 3, snapshot=snap)
    with pytest.raises(ValueError, match="past"):
        E.run_twin(wl, "bootstrap", 2, resume=snap)
