"""In-place peak memory (the paper's memory comparison, Sec. 3.1: in-place
simulation peaks at about one state).  A 28-qubit complex64 state (2 GiB)
run through every plan kind and the reductions: the caller's allocations
peak at the state itself, the library holds nothing beyond its fixed
staging ring, and the device's free memory drops by no more than the ring
plus the compiled passes' code."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W

pytestmark = pytest.mark.gpu

STAGING = 256 * 256 * 1024   # the staging ring of one device


def test_plans_and_reductions_run_in_place_at_28_qubits(gpu):
    import torch
    n = 28
    state_bytes = 8 << n
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    st = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
    st[0] = 1.0
    # the staging ring is allocated at the first pass upload
    qsv.qsv_plan_execute(qsv.qsv_plan_create(n, qsv.QSV_C64, W.qft(n)[:3], mode=qsv.PLAN_PASSES), st)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    qsv.qsv_memory_stats(reset_peak=True)
    free0 = torch.cuda.mem_get_info()[0]
    circ = W.qft(n) + W.supremacy(n, 4, seed=1)
    plans = [qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PER_GATE),
             qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_GREEDY, kmax=2),
             qsv.qsv_plan_create(n, qsv.QSV_C64, W.variational(n, 2, seed=3), mode=qsv.PLAN_GREEDY, kmax=5,
                                 use_mfma=1),
             qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES, jit=0),
             qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES, jit=1),
             qsv.qsv_plan_create(n, qsv.QSV_C64, W.variational(n, 2, seed=3), mode=qsv.PLAN_PASSES, jit=2)]
    for p in plans:
        qsv.qsv_plan_execute(p, st)
    p3 = qsv.qsv_probabilities(st, [0, n - 1, 13])
    nrm = qsv.qsv_norm2(st)
    e = qsv.qsv_expval_zz_x(st)
    torch.cuda.synchronize()
    assert abs(float(nrm.item()) - 1.0) <= 1e-4 and abs(float(p3.sum().item()) - 1.0) <= 1e-4
    assert np.isfinite(float(e.item()))
    free1 = torch.cuda.mem_get_info()[0]
    torch_peak = torch.cuda.max_memory_allocated()
    cur, peak = qsv.qsv_memory_stats()
    print("torch peak %.1f MiB over the state, library current %.1f / peak %.1f MiB, free memory drop %.1f MiB" % (
        (torch_peak - state_bytes) / 2**20, cur / 2**20, peak / 2**20, (free0 - free1) / 2**20))
    assert torch_peak <= state_bytes + (1 << 20)
    assert cur == STAGING and peak == STAGING
    assert free0 - free1 <= STAGING + (128 << 20)
