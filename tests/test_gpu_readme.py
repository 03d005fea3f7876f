"""The README's usage snippets run as written (the batched one with a small
list of instances supplied here), so the documented calls stay valid."""
import os
import re

import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_snippets_run():
    from paper_1702_05156_amd import dsgm
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert len(blocks) >= 3
    code = "\n".join(blocks)
    setup = (
        "instances = []\n"
        "for i, (T, H, W) in enumerate([(20, 48, 64), (9, 30, 40), (33, 16, 128)]):\n"
        "    f = torch.rand(T, H, W, device='cuda').to(torch.bfloat16) * 2 - 1\n"
        "    s_ = dsgm.State.empty(H, W, torch.float32)\n"
        "    dsgm.dsgm_state_init_from_frame(f[0], s_, p)\n"
        "    instances.append((f, s_))\n")
    anchor = "from paper_1702_05156_amd import tune\n"
    assert anchor in code
    code = code.replace(anchor, anchor + setup)
    scope = {"torch": torch, "dsgm": dsgm}
    exec(compile(code, "README.md", "exec"), scope)
    torch.cuda.synchronize()
    # a few of the documented results are what they say they are
    assert scope["out"]["masks"].dtype == torch.uint8
    assert scope["x"].grad is not None and scope["vi"].grad is not None
    for f, s_, m, _, c in scope["items"]:
        assert torch.equal(c.to(torch.int64), (m == 255).flatten(1).sum(1))
