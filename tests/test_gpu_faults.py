"""Out-of-memory paths, forced from the host with MC_EXPMV_FAULT=alloc:K (the K-th
allocation of a call fails, nothing is allocated): every failing call returns
MC_ERR_NO_MEMORY, frees what it had allocated (device free memory is back where
it was), leaves an existing handle usable, and a later call without the fault
gives the same estimates as a fresh handle.  No kernel sees a fault: the hook
fails the allocation before anything is launched with it."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1904_12759_amd as mc
from paper_1904_12759_amd import workloads as wl

pytestmark = pytest.mark.gpu

NO_MEMORY = 6


@pytest.fixture
def fault():
    def set_k(k):
        if k is None:
            os.environ.pop("MC_EXPMV_FAULT", None)
        else:
            os.environ["MC_EXPMV_FAULT"] = f"alloc:{k}"
    yield set_k
    os.environ.pop("MC_EXPMV_FAULT", None)


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(0)[0]


def test_create_fails_cleanly_at_every_allocation(fault):
    a = wl.grid2d(384)                     # n = 147456: tables of several MB each
    v = wl.uniform_v(a.n, 2)
    idx = np.array([0, 1000, a.n - 1])
    ref = mc.MCExpmv(a.rowptr, a.col, a.val, 0.3, 9, relabel=1)
    e0, s0 = ref.entries(v, idx, 3000)
    del ref
    f0 = _free()
    seen = 0
    for k in range(1, 200):
        fault(k)
        try:
            h = mc.MCExpmv(a.rowptr, a.col, a.val, 0.3, 9, relabel=1)
        except mc.MCError as err:
            assert err.code == NO_MEMORY, (k, err)
            seen += 1
            fault(None)
            assert _free() >= f0, (k, f0 - _free())
            continue
        fault(None)
        break
    else:
        pytest.fail("create never succeeded")
    print(f"create: allocations 1..{seen} failed cleanly, {seen + 1} succeeded", flush=True)
    assert seen >= 8
    e1, s1 = h.entries(v, idx, 3000)
    assert torch.equal(e0, e1) and torch.equal(s0, s1)


def test_entries_partials_allocation_fails_then_recovers(fault):
    a = wl.grid2d(32)
    v = wl.uniform_v(a.n, 2)
    idx = torch.arange(0, a.n, 7, device="cuda")
    h = mc.MCExpmv(a.rowptr, a.col, a.val, 0.3, 9)
    fault(1)                                   # the chunk partials of a multi-chunk run
    with pytest.raises(mc.MCError) as err:
        h.entries(v, idx, 5000)
    assert err.value.code == NO_MEMORY
    # the no-allocation entry point makes no allocation for the hook to fail
    est = torch.empty(idx.numel(), dtype=torch.float64, device="cuda")
    h.entries_noalloc(h._v(v), idx, 5000, est, None)
    fault(None)
    e1, _ = h.entries(v, idx, 5000)
    assert torch.equal(e1, est)
    fresh = mc.MCExpmv(a.rowptr, a.col, a.val, 0.3, 9)
    e2, _ = fresh.entries(v, idx, 5000)
    assert torch.equal(e1, e2)


def test_batch_create_and_isim_fail_cleanly(fault):
    ws = wl.batched_instances(count=4, nmax=2e4)
    insts = [dict(rowptr=w.a.rowptr, col=w.a.col, val=w.a.val, t=w.t, v=w.v, idx=w.idx,
                  n_walkers=64 if w.idx is None else 1000, instance_id=k)
             for k, w in enumerate(ws)]
    for k in (1, 2, 5, 11):
        fault(k)
        with pytest.raises(mc.MCError) as err:
            mc.MCBatch(insts, 3)
        assert err.value.code == NO_MEMORY
    fault(None)
    b = mc.MCBatch(insts, 3)
    b.run()
    x = torch.rand(1000, dtype=torch.float64, device="cuda")
    y = torch.rand(1000, dtype=torch.float64, device="cuda")
    want = mc.isim(x, y)
    for k in (1, 4, 9):
        fault(k)
        with pytest.raises(mc.MCError) as err:
            mc.isim(x, y)
        assert err.value.code == NO_MEMORY
    fault(None)
    assert mc.isim(x, y) == want


def test_stencil_create_fails_cleanly_at_every_allocation(fault):
    m = 24
    a = wl.grid3d(m, 1)
    fx, fy, fz, diag = wl.stencil7_faces(a, m, m, m)
    v = wl.bump_v(m, 2)
    idx = np.array([0, 5000, a.n - 1])
    ref = mc.MCExpmv.stencil7(m, m, m, fx, fy, fz, diag, 0.05, 4)
    e0, s0 = ref.entries(v, idx, 3000)
    del ref
    f0 = _free()
    seen = 0
    for k in range(1, 100):
        fault(k)
        try:
            h = mc.MCExpmv.stencil7(m, m, m, fx, fy, fz, diag, 0.05, 4)
        except mc.MCError as err:
            assert err.code == NO_MEMORY, (k, err)
            seen += 1
            fault(None)
            assert _free() >= f0, (k, f0 - _free())
            continue
        fault(None)
        break
    else:
        pytest.fail("create_stencil7 never succeeded")
    # flags, host flag, counters, row records, thresholds, d64, d32, the face staging
    assert seen >= 8
    e1, s1 = h.entries(v, idx, 3000)
    assert torch.equal(e0, e1) and torch.equal(s0, s1)
