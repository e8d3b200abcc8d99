"""sim_segsort_noalloc (the allocation-free segmented sort) against sim_segsort,
through the C-ABI: two calls in a row on the library's shared scratch array,
the second on a smaller input, each bit-exact against the allocating entry
point (integer permutation and offsets)."""
import numpy as np
import pytest

from paper_2603_25068_amd import workloads as W

pytestmark = pytest.mark.gpu


def _keys(rng, n, nseg):
    seg = rng.integers(0, nseg, n).astype(np.int32)
    pos = rng.choice(np.float32([0.0, 1.5, 2.25, 100.0, 7.0]), n) + rng.integers(0, 3, n).astype(np.float32)
    seq = rng.integers(0, 50, n).astype(np.int32)
    return seg, pos, seq


def test_noalloc_sort_matches_allocating_sort_twice():
    import torch
    from paper_2603_25068_amd.sim import Simulator
    s = Simulator(W.tg_toy())
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(17)
    for n, nseg in ((40000, 3000), (5000, 41)):
        seg, pos, seq = _keys(rng, n, nseg)
        tseg, tpos, tseq = (torch.from_numpy(a).to(dev) for a in (seg, pos, seq))
        perm_ref, off_ref = s.segsort(tseg, tpos, tseq, nseg)
        perm = torch.full((n,), -7, dtype=torch.int32, device=dev)
        off = torch.full((nseg + 1,), -7, dtype=torch.int32, device=dev)
        s.segsort_noalloc(tseg, tpos, tseq, nseg, perm, off)
        assert torch.equal(perm, perm_ref), f"n={n}: permutation differs from sim_segsort"
        assert torch.equal(off, off_ref), f"n={n}: offsets differ from sim_segsort"
        # and both are the (segment, position desc, sequence, index) order
        ref = np.lexsort((np.arange(n), seq, -pos, seg))
        assert np.array_equal(perm.cpu().numpy(), ref)


def test_noalloc_sort_status_flag_and_limits():
    import torch
    from paper_2603_25068_amd.sim import Simulator, SimError, SIM_EINVAL
    s = Simulator(W.tg_toy())
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    # asynchronous form: the flag is written in stream order
    n, nseg = 3000, 7
    seg, pos, seq = _keys(rng, n, nseg)
    tseg, tpos, tseq = (torch.from_numpy(a).to(dev) for a in (seg, pos, seq))
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    off = torch.empty(nseg + 1, dtype=torch.int32, device=dev)
    status = torch.full((1,), 9, dtype=torch.int32, device=dev)
    s.segsort_noalloc(tseg, tpos, tseq, nseg, perm, off, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert np.array_equal(perm.cpu().numpy(), np.lexsort((np.arange(n), seq, -pos, seg)))
    # a segment longer than the LDS sort holds (2,048 keys): the kernel's own check reports it
    big = np.zeros(2100, np.int32)
    tb = torch.from_numpy(big).to(dev)
    tp = torch.zeros(2100, dtype=torch.float32, device=dev)
    perm2 = torch.empty(2100, dtype=torch.int32, device=dev)
    off2 = torch.empty(2, dtype=torch.int32, device=dev)
    s.segsort_noalloc(tb, tp, tb, 1, perm2, off2, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 1
    # sizes beyond the fixed array are rejected on the host before any launch
    with pytest.raises(SimError) as e:
        s.segsort_noalloc(tseg, tpos, tseq, (1 << 20) + 1, perm, off)
    assert e.value.code == SIM_EINVAL
