"""The launch-shape autotuner: candidates timed, the best cached, and results
independent of the shape it picks."""
import json

import pytest
import torch

from tests import gpu_util as G

pytestmark = pytest.mark.gpu

dsgm = pytest.importorskip("paper_1702_05156_amd.dsgm")
tune = pytest.importorskip("paper_1702_05156_amd.tune")


def test_tune_forward_caches_and_applies(tmp_path, monkeypatch):
    monkeypatch.setenv("DSGM_TUNE_CACHE", str(tmp_path / "tune.json"))
    T, H, W = 40, 64, 512
    p = dsgm.dsgm_params_default(2.0)
    fr, st = G.device_case(41, T, H, W, torch.float32, torch.float32)
    before = st.clone()
    r = tune.tune_forward(fr, st, p, reps=2)
    assert len(r["candidates"]) == 9
    for a, b in zip(st.planes(), before.planes()):
        assert torch.equal(a, b)  # the caller's state is untouched
    key = tune.forward_key(fr, st)
    cache = json.loads((tmp_path / "tune.json").read_text())
    assert cache[key]["block"] == r["block"] and cache[key]["vector"] == r["vector"]
    ref = dsgm.forward(fr, st.clone(), p)
    with tune.tuned(key) as best:
        assert best["vector"] == r["vector"]
        got = dsgm.forward(fr, st.clone(), p)
    assert torch.equal(got["masks"], ref["masks"])
