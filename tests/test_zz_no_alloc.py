"""GPU tests of mc_expmv_entries_noalloc, the entry point that allocates nothing
(its chunk partials in a static device array): through the C ABI it must give
exactly mc_expmv_entries' estimates, on two calls in a row (the second smaller),
reject requests beyond its fixed scratch before enqueuing anything, and leave
the device's free memory unchanged."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1904_12759_amd as mc
from paper_1904_12759_amd import workloads as wl

pytestmark = pytest.mark.gpu

SCRATCH = 1 << 20          # MC_NOALLOC_SCRATCH_DOUBLES


def _case(fp32):
    a = wl.grid2d(24)
    v = wl.uniform_v(a.n, 2)
    h = mc.MCExpmv(a.rowptr, a.col, a.val, 0.4, 321, fp32=fp32)
    dev = torch.device("cuda", 0)
    vt = torch.as_tensor(v, dtype=torch.float32 if fp32 else torch.float64, device=dev)
    return a, h, vt, dev


@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_equals_entries_two_calls(fp32):
    a, h, vt, dev = _case(fp32)
    rng = np.random.default_rng(7)
    # first call: 300 entries x 5000 walkers (several chunks, ragged last chunk);
    # second call: fewer entries and walkers, with a duplicate index
    for k, nwalk in ((300, 5000), (37, 1777)):
        idx = torch.as_tensor(rng.choice(a.n, k, replace=True), device=dev)
        e0 = torch.empty(k, dtype=torch.float64, device=dev)
        s0 = torch.empty(k, dtype=torch.float64, device=dev)
        e1 = torch.full((k,), float("nan"), dtype=torch.float64, device=dev)
        s1 = torch.full((k,), float("nan"), dtype=torch.float64, device=dev)
        h.entries(vt, idx, nwalk, est=e0, stderr=s0)
        h.entries_noalloc(vt, idx, nwalk, e1, s1)
        print(f"noalloc fp32={fp32} k={k} walkers={nwalk}: "
              f"max |diff| {float((e1 - e0).abs().max()):.3g}", flush=True)
        assert torch.equal(e0, e1)
        assert torch.equal(s0, s1)
        st = h.stats()
        assert st["walkers"] == k * nwalk


def test_noalloc_single_chunk_and_empty():
    a, h, vt, dev = _case(False)
    idx = torch.as_tensor([0, 5, 5, a.n - 1], device=dev)
    e0, s0 = h.entries(vt, idx, 300)
    e1 = torch.empty(4, dtype=torch.float64, device=dev)
    s1 = torch.empty(4, dtype=torch.float64, device=dev)
    h.entries_noalloc(vt, idx, 300, e1, s1)
    assert torch.equal(e0, e1) and torch.equal(s0, s1)
    empty = torch.empty(0, dtype=torch.int64, device=dev)
    out = torch.empty(0, dtype=torch.float64, device=dev)
    h.entries_noalloc(vt, empty, 300, out, None)


def test_noalloc_rejects_requests_beyond_scratch():
    a, h, vt, dev = _case(False)
    chunk = 512                                       # FP64 weights
    nwalk = 400 * chunk                               # 400 chunks per entry
    k = SCRATCH // (3 * 400) + 1                      # one entry too many
    idx = torch.zeros(k, dtype=torch.int64, device=dev)
    est = torch.full((k,), -1.0, dtype=torch.float64, device=dev)
    with pytest.raises(mc.MCError) as err:
        h.entries_noalloc(vt, idx, nwalk, est, None)
    assert err.value.code == 10                      # MC_ERR_TOO_LARGE
    torch.cuda.synchronize()
    assert bool((est == -1.0).all())                  # nothing was enqueued
    # exactly at the limit it runs, and equals entries
    k = SCRATCH // (3 * 400)
    idx = torch.as_tensor(np.arange(k) % a.n, device=dev)
    e1 = torch.empty(k, dtype=torch.float64, device=dev)
    h.entries_noalloc(vt, idx, nwalk, e1, None)
    e0, _ = h.entries(vt, idx, nwalk)
    assert torch.equal(e0, e1)


def test_noalloc_leaves_free_memory_unchanged():
    """A fresh handle's first mc_expmv_entries with many chunk partials allocates
    them (free memory drops); mc_expmv_entries_noalloc on another fresh handle does
    not."""
    a, h, vt, dev = _case(False)
    k, nwalk = 200, 512 * 1000                        # 200 x 1000 chunks: 4.8 MB of partials
    idx = torch.as_tensor(np.arange(k) % a.n, device=dev)
    est = torch.empty(k, dtype=torch.float64, device=dev)
    h.entries(vt, idx, 1000, est=est)                 # load the kernels once
    h.entries_noalloc(vt, idx, 1000, est, None)
    h2 = mc.MCExpmv(a.rowptr, a.col, a.val, 0.4, 321)
    torch.cuda.synchronize()
    f0 = torch.cuda.mem_get_info(dev)[0]
    h2.entries_noalloc(vt, idx, nwalk, est, None)
    torch.cuda.synchronize()
    f1 = torch.cuda.mem_get_info(dev)[0]
    h3 = mc.MCExpmv(a.rowptr, a.col, a.val, 0.4, 321)
    big = torch.as_tensor(np.arange(1000) % a.n, device=dev)   # 24 MB of partials
    est3 = torch.empty(1000, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    f2 = torch.cuda.mem_get_info(dev)[0]
    h3.entries(vt, big, nwalk, est=est3)
    torch.cuda.synchronize()
    f3 = torch.cuda.mem_get_info(dev)[0]
    print(f"free memory change: noalloc {f1 - f0} B, entries {f3 - f2} B", flush=True)
    assert f1 == f0
    assert f3 < f2                                    # the check sees a 24 MB allocation
