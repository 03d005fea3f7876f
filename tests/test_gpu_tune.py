"""The launch-shape autotuner: candidates timed, the best cached, and results
independent of the shape it picks."""
import json

import pytest
import torch

from synth import device as sdev
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


def test_tune_batched_picks_a_width_and_results_do_not_depend_on_it(tmp_path, monkeypatch):
    """The batched autotuner times every tile width the instances allow; the
    plan made with the chosen width gives the same masks and state as the
    default plan."""
    monkeypatch.setenv("DSGM_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_1702_05156_amd import tune
    p = dsgm.dsgm_params_default(2.0)
    shapes = [(20, 16, 64), (7, 8, 128), (33, 24, 32)]

    def make():
        items = []
        for i, (T, H, W) in enumerate(shapes):
            fr = sdev.frames(80 + i, T, H, W, torch.bfloat16)
            st = dsgm.State(*sdev.state(80 + i, H, W, torch.float32))
            items.append((fr, st, torch.empty((T, H, W), dtype=torch.uint8, device="cuda"), None))
        return items
    best = tune.tune_batched(make(), p)
    assert best["vector"] in (1, 2, 4) and len(best["candidates"]) >= 2
    assert tune.lookup(tune.batched_key(make()))["vector"] == best["vector"]
    a, b = make(), make()
    dsgm.Batch(a).run(p)
    dsgm.Batch(b, vector=best["vector"]).run(p)
    torch.cuda.synchronize()
    for (_, sa, ma, _), (_, sb, mb, _) in zip(a, b):
        assert torch.equal(ma, mb)
        for u, v in zip(sa.planes(), sb.planes()):
            assert torch.equal(u, v)
