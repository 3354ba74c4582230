"""The no-allocation probabilities entry point (for callers that cannot
allocate) against qsv_probabilities, through the C ABI: two calls in a row,
the second on a smaller input, both with decompositions that use the
library's partial array and ones that write the output directly."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_noalloc_probabilities_match(gpu, dt):
    import torch
    t = torch.complex64 if dt == "c64" else torch.complex128
    cases = [(20, [1, 0]), (16, [3, 12, 7]), (18, [17]), (12, list(range(12)))]
    for n, qs in cases:   # each call after a larger (or different) one
        st = torch.from_numpy(W.random_state(n, n)).to(t).cuda()
        want = qsv.qsv_probabilities(st, qs)
        out = torch.full((1 << len(qs),), -1.0, dtype=torch.float64, device="cuda")
        qsv.qsv_probabilities_noalloc(st, qs, out)
        torch.cuda.synchronize()
        # the same kernels in the same order: equal bit for bit
        assert torch.equal(out, want), (n, qs)
    with pytest.raises(ValueError):
        qsv.qsv_probabilities_noalloc(st, qs, None)
