"""The streaming step (one frame per call) under HIP graph capture.

A live source delivers one frame at a time, so a caller captures the per-frame
call once, with a fixed input slot and fixed outputs, and replays the graph for
every frame after copying the frame into the slot.  dsgm_forward (T = 1) and
dsgm_forward_warped enqueue only their kernels (no allocation, no memset, no
synchronisation), so the captured step must give, frame after frame, exactly
the results of the eager calls.  Every replay is checked, with eager work and
synchronisations between the replays.
"""
import numpy as np
import pytest
import torch

from tests import gpu_util as G

pytestmark = pytest.mark.gpu

from paper_1702_05156_amd import dsgm


@pytest.mark.parametrize("in_dtype,acc_dtype", [(torch.float64, torch.float64),
                                                (torch.bfloat16, torch.float32)])
def test_streaming_step_graph_replays_equal_eager(in_dtype, acc_dtype):
    T, H, W = 12, 40, 96
    p = dsgm.dsgm_params_default(2.0)
    fr, st0 = G.device_case(61, T, H, W, in_dtype, acc_dtype)
    # eager: one call per frame
    st = st0.clone()
    want_m = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    want_bg = torch.empty((T, H, W), dtype=acc_dtype, device="cuda")
    for t in range(T):
        dsgm.dsgm_forward(fr[t:t + 1], st, p, want_m[t:t + 1], want_bg[t:t + 1])
    torch.cuda.synchronize()
    want_st = st

    # captured: a fixed slot, fixed outputs, the state updated in place by
    # every replay (capture itself runs nothing)
    slot = torch.empty((1, H, W), dtype=in_dtype, device="cuda")
    m = torch.empty((1, H, W), dtype=torch.uint8, device="cuda")
    bg = torch.empty((1, H, W), dtype=acc_dtype, device="cuda")
    gst = st0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        dsgm.dsgm_forward(slot, gst, p, m, bg)
    torch.cuda.synchronize()
    for a, b in zip(gst.planes(), st0.planes()):
        assert torch.equal(a, b)
    for t in range(T):
        slot.copy_(fr[t:t + 1])
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(m[0], want_m[t]), t
        assert torch.equal(bg[0], want_bg[t]), t
        torch.ones(1000, device="cuda").sum().item()  # eager work between replays
    for a, b in zip(gst.planes(), want_st.planes()):
        assert torch.equal(a, b)


def test_warped_steps_graphs_replay_equal_eager():
    """The motion-compensated step ping-pongs two model buffers; its homography
    is a launch argument, so each frame's step is captured with its matrix."""
    T, H, W = 10, 36, 80
    p = dsgm.dsgm_params_default(2.0)
    fr, st0 = G.device_case(62, T, H, W)
    rng = np.random.default_rng(7)
    maps = []
    for _ in range(T):
        mt = np.eye(3)
        mt[0, 2], mt[1, 2] = rng.uniform(-1.5, 1.5, size=2)
        mt[0, 1], mt[1, 0] = rng.uniform(-0.01, 0.01, size=2)
        maps.append(mt)
    # eager
    bufs = [st0.clone(), dsgm.State.empty(H, W)]
    want = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
    for t in range(T):
        dsgm.dsgm_forward_warped(fr[t], bufs[t % 2], bufs[1 - t % 2], p, maps[t], want[t])
    torch.cuda.synchronize()
    want_st = bufs[T % 2]

    # the homography is a host argument of the launch, so a captured step
    # holds the matrix it was captured with: capture one graph per frame
    gb = [st0.clone(), dsgm.State.empty(H, W)]
    slot = torch.empty((H, W), dtype=torch.float64, device="cuda")
    m = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graphs = []
    for t in range(T):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            dsgm.dsgm_forward_warped(slot, gb[t % 2], gb[1 - t % 2], p, maps[t], m)
        graphs.append(g)
    torch.cuda.synchronize()
    # capture runs nothing: the first buffer still holds the start
    for a, b in zip(gb[0].planes(), st0.planes()):
        assert torch.equal(a, b)
    for t in range(T):
        slot.copy_(fr[t])
        torch.cuda.synchronize()
        graphs[t].replay()
        torch.cuda.synchronize()
        assert torch.equal(m, want[t]), t
        torch.ones(1000, device="cuda").sum().item()
    for a, b in zip(gb[T % 2].planes(), want_st.planes()):
        assert torch.equal(a, b)
