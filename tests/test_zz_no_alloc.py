"""GPU: lt_transfer_noalloc (the transfer's scratch in the library's static
device array, no allocation) against lt_transfer on the same mapping: equal
bit for bit, on two calls in a row whose second input is smaller (the
static array still holds the first call's contents), with the registered
allocator capped at what the tree already holds; LT_ERR_STATE before any
mapping and LT_ERR_ARG beyond 2^25 leaves."""
import numpy as np
import pytest

from paper_2306_06744_amd import synth

from gpu_util import adapt_both, both

pytestmark = pytest.mark.gpu


def _cycle_tree(dim, d_max, seed, cycles):
    g, o = both(dim, 2, d_max)
    for c in range(cycles):
        adapt_both(g, o, synth.random_flags(seed + c, o.size(), 0.3, 0.4))
        g.balance()
        o.balance()
    return g


def test_noalloc_transfer_matches_transfer():
    import torch
    import paper_2306_06744_amd as lt
    a = lt.TorchAllocator()
    lt.set_allocator(a)
    try:
        big = _cycle_tree(3, 6, 800, 4)
        small = _cycle_tree(3, 4, 900, 2)
        cases = [(big, 3, 5), (small, 3, 5), (_cycle_tree(2, 8, 950, 3), 5, 3)]
        for i, (t, p, nvar) in enumerate(cases):
            n, n_old, _ = t.sizes()
            print("case", i, n_old, "->", n, "p", p, flush=True)
            npts = (p + 1) ** t.dim
            u_old = torch.from_numpy(synth.random_solution(10 + i, nvar, npts, n_old + 3)).cuda()
            ref = t.transfer(p, u_old)                       # computes the mapping
            out = torch.full((nvar, npts, n + 5), float("nan"), dtype=torch.float64, device="cuda")
            a.limit = a.held                                  # nothing more may be allocated
            t.transfer_noalloc(p, u_old, out)
            torch.cuda.synchronize()
            a.limit = None
            assert torch.equal(out[:, :, :n], ref), f"case {i} differs"
            assert torch.isnan(out[:, :, n:]).all()
    finally:
        lt.set_allocator(None)


def test_noalloc_transfer_errors():
    import torch
    import paper_2306_06744_amd as lt
    t = lt.Tree.uniform(3, 2, 5, depth=3)
    u = torch.zeros((1, 8, t.size()), dtype=torch.float64, device="cuda")
    with pytest.raises(lt.LtError) as ei:
        t.transfer_noalloc(1, u, u.clone())
    assert ei.value.status == 7
    big = lt.Tree.uniform(2, 0, 13, depth=13)               # 2^26 leaves
    big.adapt(torch.zeros(big.size(), dtype=torch.int8, device="cuda"))
    big.map()
    with pytest.raises(lt.LtError) as ei:
        big.transfer_noalloc(1, u, u.clone())
    assert ei.value.status == 1 and "2^25" in str(ei.value)
