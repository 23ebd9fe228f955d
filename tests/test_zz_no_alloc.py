"""conv_step_static, the allocation-free conv_step (static device scratch instead of a workspace),
checked through the C ABI against conv_step on the same inputs: two calls in a row, the second
smaller, so the second runs on the scratch the first left behind."""
import numpy as np
import pytest

from paper_1711_00289_amd import binding as B
from paper_1711_00289_amd import soundings as S


@pytest.mark.gpu
def test_static_step_matches_conv_step_on_two_calls():
    import torch

    grid = S.grid_1deg()
    # The 55,296-column 1-degree grid, then 4,097 of its columns (a ragged tail, tropical rows):
    # every output element is compared bit for bit with conv_step's.
    for cols in (None, np.arange(288 * 80, 288 * 80 + 4097)):
        st = grid if cols is None else S.subset(grid, cols)
        n = st["ncol"]
        print(f"conv_step_static vs conv_step: {n} columns x 30 levels", flush=True)
        dev = B.to_device(st)
        conv = B.Conv(n, 30)
        d_ref, s_ref = conv.step(dev)
        d = B.alloc_deep(torch, "cuda", 30, n)
        s = B.alloc_shallow(torch, "cuda", 30, n)
        for t in (*d.values(), *s.values()):
            t.fill_(7)  # every element must be written
        assert B.step_static(dev, n, 30, d, s) == B.CONV_OK
        torch.cuda.synchronize()
        for f in d:
            assert torch.equal(d[f], d_ref[f]), f"deep {f} ({n} columns)"
        for f in s:
            assert torch.equal(s[f], s_ref[f]), f"shallow {f} ({n} columns)"
        assert int((d["status"] == 0).sum()) > 0 and int((s["status"] == 0).sum()) > 0
