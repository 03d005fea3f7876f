"""GPU batched forward: one persistent launch over many uneven instances.

Every instance's masks, bg and final state must be bit-identical to a
single-instance dsgm_forward on the same inputs (same kernel body, same
order of operations), and FP64 instances bit-identical to the oracle.  The
launch is captured into a graph and replayed; every replay is checked against
the eager result.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import device as sdev
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

from paper_1702_05156_amd import dsgm

SHAPES = [(40, 16, 64), (3, 8, 8), (120, 4, 256), (1, 1, 4), (17, 24, 32), (64, 32, 128),
          (0, 8, 16), (9, 0, 16), (33, 7, 12), (250, 2, 8)]


def _make(shapes, in_dtype, acc_dtype, bg=True, seed0=300):
    items, ref_inputs = [], []
    for i, (T, H, W) in enumerate(shapes):
        fr = sdev.frames(seed0 + i, T, H, W, in_dtype) if T * H * W else \
            torch.zeros((T, H, W), dtype=in_dtype, device="cuda")
        st = dsgm.State(*sdev.state(seed0 + i, H, W, acc_dtype)) if H * W else dsgm.State.empty(H, W, acc_dtype)
        masks = torch.empty((T, H, W), dtype=torch.uint8, device="cuda")
        b = torch.empty((T, H, W), dtype=acc_dtype, device="cuda") if bg else None
        items.append((fr, st, masks, b))
        ref_inputs.append((fr, st.clone()))
    return items, ref_inputs


@pytest.mark.parametrize("in_dtype,acc_dtype", [(torch.float64, torch.float64),
                                                (torch.float32, torch.float32),
                                                (torch.bfloat16, torch.float32)])
def test_batched_equals_single_calls(in_dtype, acc_dtype):
    p = dsgm.dsgm_params_default(2.0)
    items, refs = _make(SHAPES, in_dtype, acc_dtype)
    batch = dsgm.Batch(items)
    assert batch.plan.vector == (4 if in_dtype == torch.bfloat16 else 2)  # measured defaults
    batch.run(p)
    torch.cuda.synchronize()
    for (fr, st, masks, bg), (fr0, st0) in zip(items, refs):
        T, H, W = fr.shape
        if T * H * W == 0:
            continue
        o = dsgm.forward(fr0, st0, p, bg=True)
        torch.cuda.synchronize()
        assert torch.equal(masks, o["masks"]), (T, H, W)
        assert torch.equal(bg, o["bg"])
        for a, b in zip(st.planes(), st0.planes()):
            assert torch.equal(a, b)


def test_batched_ragged_widths_and_oracle():
    """An odd width forces one pixel per lane for the whole batch; FP64 results
    are checked against the oracle instance by instance."""
    shapes = [(21, 5, 13), (30, 9, 40), (7, 3, 7)]
    p = dsgm.dsgm_params_default(2.0)
    items, _ = _make(shapes, torch.float64, torch.float64, seed0=400)
    batch = dsgm.Batch(items)
    assert batch.plan.vector == 1
    batch.run(p)
    torch.cuda.synchronize()
    for i, ((fr, st, masks, bg), (T, H, W)) in enumerate(zip(items, shapes)):
        x, s0 = G.host_case(400 + i, T, H, W)
        ref = oracle.forward(x, s0, G.oracle_params(p))
        G.assert_bit_exact(f"masks[{i}]", G.flat(masks), ref["masks"])
        G.assert_bit_exact(f"bg[{i}]", G.flat(bg), ref["bg"])
        hs = G.state_to_host(st)
        for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
            G.assert_bit_exact(f"{k}[{i}]", hs[k], ref[k])


@pytest.mark.parametrize("wr,mr", [(1, 1), (0, 1), (1, 0)])
def test_batched_other_rules_f64_oracle(wr, mr):
    """The appendix's weights and its printed mask rule (a compiled variant of
    the persistent kernel) on a batch, FP64, every instance against the oracle."""
    shapes = [(25, 6, 16), (40, 9, 32), (3, 4, 8)]
    p = dsgm.dsgm_params_default(2.0, mr)
    p.weight_rule = wr
    items, _ = _make(shapes, torch.float64, torch.float64, seed0=450)
    batch = dsgm.Batch(items)
    batch.run(p)
    torch.cuda.synchronize()
    for i, ((fr, st, masks, bg), (T, H, W)) in enumerate(zip(items, shapes)):
        x, s0 = G.host_case(450 + i, T, H, W)
        ref = oracle.forward(x, s0, G.oracle_params(p))
        G.assert_bit_exact(f"masks[{i}]", G.flat(masks), ref["masks"])
        G.assert_bit_exact(f"bg[{i}]", G.flat(bg), ref["bg"])
        hs = G.state_to_host(st)
        for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
            G.assert_bit_exact(f"{k}[{i}]", hs[k], ref[k])


def test_batched_lpt_order_and_plan():
    p = dsgm.dsgm_params_default(2.0)
    items, _ = _make(SHAPES, torch.float32, torch.float32)
    batch = dsgm.Batch(items)
    P = batch.plan.vector
    assert P == 2
    groups = [(H * W // P + 63) // 64 for T, H, W in SHAPES if T * H * W]
    assert batch.plan.n_items == sum(groups)
    assert batch.plan.total_elements == sum(T * H * W for T, H, W in SHAPES)
    assert batch.plan.grid >= 256
    # item table: costs non-increasing
    hdr = 256
    ninst = len(SHAPES)
    inst_bytes = ((ninst * 136 + 255) // 256) * 256  # sizeof(BatchInst) = 136
    raw = batch.plan_buffer.cpu().numpy()
    it = raw[hdr + inst_bytes: hdr + inst_bytes + 16 * batch.plan.n_items].view(np.int32).reshape(-1, 4)
    T = np.array([s[0] for s in SHAPES])
    cost = T[it[:, 0]] * it[:, 2]
    assert np.all(np.diff(cost) <= 0)
    del p


def test_batched_graph_capture_replays():
    p = dsgm.dsgm_params_default(2.0)
    items, refs = _make(SHAPES, torch.float32, torch.float32, seed0=500)
    init = [st.clone() for _, st, _, _ in items]
    batch = dsgm.Batch(items)
    # eager reference
    batch.run(p)
    torch.cuda.synchronize()
    want = [(m.clone(), b.clone(), tuple(x.clone() for x in st.planes())) for _, st, m, b in items]

    def restore():
        for (_, st, m, b), s0 in zip(items, init):
            for a, c in zip(st.planes(), s0.planes()):
                a.copy_(c)
            m.zero_()
            b.zero_()

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        batch.run(p)
    torch.cuda.synchronize()
    for rep in range(3):
        restore()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for (_, st, m, b), (wm, wb, ws) in zip(items, want):
            assert torch.equal(m, wm), rep
            assert torch.equal(b, wb), rep
            for a, c in zip(st.planes(), ws):
                assert torch.equal(a, c), rep
        # some eager work between replays
        torch.ones(1000, device="cuda").sum().item()


@pytest.mark.parametrize("in_dtype,acc_dtype", [(torch.bfloat16, torch.float32),
                                                (torch.float64, torch.float64)])
def test_batched_foreground_counts(in_dtype, acc_dtype):
    """Per-frame foreground counts of the instances that ask for them, equal to
    the count of 255s in their masks (exact integers), nothing written for the
    others; every replay of a captured launch clears and recounts them."""
    p = dsgm.dsgm_params_default(2.0)
    items, _ = _make(SHAPES, in_dtype, acc_dtype, bg=False, seed0=700)
    sentinel = -7
    counts = [torch.full((T,), sentinel, dtype=torch.int32, device="cuda") if i % 3 != 1 else None
              for i, (T, H, W) in enumerate(SHAPES)]
    items = [it[:3] + (None, c) for it, c in zip(items, counts)]
    init = [st.clone() for _, st, *_ in items]
    batch = dsgm.Batch(items)
    assert batch.plan.has_counts == 1

    def check(tag):
        for i, ((fr, st, masks, _, c), (T, H, W)) in enumerate(zip(items, SHAPES)):
            if c is None:
                continue
            if T * H * W == 0:
                # no work: the counters are left as they were
                assert bool((c == sentinel).all()), (tag, i)
                continue
            want = (masks.view(T, -1) == 255).sum(dim=1).to(torch.int32)
            assert torch.equal(c, want), (tag, i, c[:8].tolist(), want[:8].tolist())
            assert int(want.sum()) > 0

    batch.run(p)
    torch.cuda.synchronize()
    check("eager")

    def restore():
        for (_, st, m, _, _), s0 in zip(items, init):
            for a, b in zip(st.planes(), s0.planes()):
                a.copy_(b)
            m.zero_()

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        batch.run(p)
    torch.cuda.synchronize()
    for rep in range(3):
        restore()
        for c, (T, H, W) in zip(counts, SHAPES):
            if c is not None and T * H * W:
                c.fill_(123456)  # stale values that the launch must clear
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        check(f"replay {rep}")
        torch.ones(1000, device="cuda").sum().item()


def test_batched_rejects_mixed_dtypes():
    items, _ = _make([(4, 4, 8)], torch.float32, torch.float32)
    items2, _ = _make([(4, 4, 8)], torch.float64, torch.float64)
    with pytest.raises(ValueError):
        dsgm.Batch(items + items2)


@pytest.mark.slow
def test_full_size_batched_sampled():
    """The benchmark's batched workload: 512 instances of log-uniform size
    (60 G elements, BF16 frames, FP32 state, masks only) in one graph-captured
    persistent launch.  For 16 instances (the largest, the smallest and 14 at
    random) 64 random pixels are replayed by the FP64 oracle on the same (BF16)
    frames and (FP32-grid) initial state.  Pixels none of whose decisions is
    within 1e-5 of its threshold must have identical masks and ages and the final
    state within 1e-5; they must be the large majority."""
    import bench
    shapes = bench.batch_shapes()
    p = dsgm.dsgm_params_default(2.0)
    items = []
    for i, (T, H, W) in enumerate(shapes):
        fr = sdev.frames(bench.batch_seed(i), T, H, W, torch.bfloat16)
        st = dsgm.State(*sdev.state(bench.batch_seed(i), H, W, torch.float32))
        items.append((fr, st, torch.empty((T, H, W), dtype=torch.uint8, device="cuda"), None))
    batch = dsgm.Batch(items)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        batch.run(p)
    g.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    sizes = np.array([t * h * w for t, h, w in shapes])
    pick = set(rng.choice(len(shapes), 14, replace=False).tolist()) | {int(sizes.argmax()), int(sizes.argmin())}
    op = G.oracle_params(p)
    for i in sorted(pick):
        T, H, W = shapes[i]
        fr, st, masks, _ = items[i]
        pix = np.sort(rng.choice(H * W, 64, replace=False))
        x, s0 = G.host_case(bench.batch_seed(i), T, H, W, torch.bfloat16, torch.float32, pix=pix)
        ref = oracle.forward(x, s0, op, margins=True)
        pt = torch.as_tensor(pix, device="cuda")
        got = masks.view(T, -1)[:, pt].cpu().numpy()
        # pixels none of whose FP64 decisions is within 1e-5 of its threshold
        # cannot be decided differently by FP32 arithmetic: exact masks there
        clear = np.abs(ref["margins"]).min(axis=(0, 2)) > 1e-5
        assert clear.mean() > 0.8, (i, clear.mean())
        G.assert_bit_exact(f"masks[{i}]", got[:, clear], ref["masks"][:, clear])
        hs = G.state_to_host(st)
        for k in ("mean_a", "var_a", "mean_c", "var_c"):
            err = np.abs(hs[k][pix][clear] - ref[k][clear])
            assert np.max(err, initial=0.0) <= 1e-5 * max(1.0, float(np.max(np.abs(ref[k])))), (i, k)
        for k in ("age_a", "age_c"):
            G.assert_bit_exact(f"{k}[{i}]", hs[k][pix][clear], ref[k][clear])
    del items, batch, g
    torch.cuda.empty_cache()


def test_full_size_batched_fp64_form_chunk_sampled_bit_exact():
    """The batched benchmark's FP64 form: its first launch (163 instances,
    129 GB of FP64 frames holding the BF16 values, FP64 state from the FP32
    initial state, masks and per-frame foreground counts).  For 16 instances
    (the largest and smallest of the launch and 14 at random) 64 random pixels
    are replayed by the oracle: masks and final state bit-identical; every
    instance's counters equal the 255s of its masks."""
    import bench
    torch.cuda.empty_cache()
    shapes = bench.batch_shapes()
    idx = bench.fp64_chunks(shapes)[0]
    p = dsgm.dsgm_params_default(2.0)
    st0 = {i: dsgm.State(*sdev.state(bench.batch_seed(i), shapes[i][1], shapes[i][2], torch.float32))
           for i in idx}
    items = bench._batch_items(shapes, idx, dsgm, sdev, torch, torch.float64, torch.float64, st0)
    dsgm.Batch(items).run(p)
    torch.cuda.synchronize()
    assert bench._counts_exact(items, torch)
    rng = np.random.default_rng(4)
    sizes = np.array([shapes[i][0] * shapes[i][1] * shapes[i][2] for i in idx])
    pick = set(rng.choice(len(idx), 14, replace=False).tolist()) | {int(sizes.argmax()), int(sizes.argmin())}
    op = G.oracle_params(p)
    for j in sorted(pick):
        i = idx[j]
        T, H, W = shapes[i]
        _, st, masks, _, _ = items[j]
        pix = np.sort(rng.choice(H * W, 64, replace=False))
        x, s0 = G.host_case(bench.batch_seed(i), T, H, W, torch.bfloat16, torch.float32, pix=pix)
        ref = oracle.forward(x, s0, op, bg=False, codes=False)
        pt = torch.as_tensor(pix, device="cuda")
        G.assert_bit_exact(f"masks[{i}]", masks.view(T, -1)[:, pt].cpu().numpy(), ref["masks"])
        hs = G.state_to_host(st)
        for k in ("mean_a", "var_a", "mean_c", "var_c", "age_a", "age_c"):
            G.assert_bit_exact(f"{k}[{i}]", hs[k][pix], ref[k])
    del items, st0
    torch.cuda.empty_cache()
