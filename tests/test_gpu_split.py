"""GPU: split-precision transfer (precision=1: dense operators on BF16 matrix
cores, every operand split in three BF16 terms, FP32 accumulation, FP64
cell-mean correction) against the FP64 oracle.

Bar, per class of the mapping: refined and fused elements each within 2e-6
relative L2 (and in the largest error relative to the class's largest
value); every new element's cell mean (its Gauss-Legendre quadrature mean)
within 1e-13 of the oracle's, relative to the RMS of the field; copied
elements bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth

from gpu_util import adapt_both, assert_same_tree, assert_transfer, both, rel_l2

pytestmark = pytest.mark.gpu


def cell_means(u, dim, p):
    _, w = oracle.gauss_legendre(p + 1)
    W = np.ones(1)
    for _ in range(dim):
        W = np.kron(w, W)
    W = W / W.sum()
    return np.einsum("i,vie->ve", W, u)


@pytest.mark.parametrize("dim,p,dmax", [(3, 3, 5), (2, 7, 7)])
def test_split_transfer_random_cycles(dim, p, dmax):
    import torch
    print("split", dim, p, dmax, flush=True)
    g, o = both(dim, 2, dmax)
    nvar = 5 if dim == 3 else 4
    for c in range(4):
        adapt_both(g, o, synth.random_flags(300 + c + dim, o.size(), 0.3, 0.45))
        g.balance()
        o.balance()
        assert_same_tree(g, o, f"cycle {c}")
        n_old = o.old_size()
        u_old = synth.random_solution(40 + c, nvar, (p + 1) ** dim, n_old)
        ref = o.transfer(p, u_old)
        got = g.transfer(p, torch.from_numpy(u_old).cuda(), precision=1).cpu().numpy()
        err = rel_l2(got, ref)
        rms = np.sqrt(np.mean(ref ** 2))
        dmean = np.abs(cell_means(got, dim, p) - cell_means(ref, dim, p)).max() / rms
        src, kind = o.map()
        copies = kind == 0
        print(f"cycle {c}: rel L2 {err:.3e}, max mean error {dmean:.3e}, "
              f"refined {(kind > 0).sum()}, fused {(kind < 0).sum()}", flush=True)
        assert_transfer(got, ref, kind, 2e-6, f"split cycle {c}")
        assert dmean <= 1e-13
        assert np.array_equal(got[:, :, copies], ref[:, :, copies])


def test_split_rejects_other_degrees():
    import torch
    import paper_2306_06744_amd as lt
    g, o = both(3, 2, 4)
    adapt_both(g, o, synth.random_flags(1, o.size(), 0.3, 0.0))
    u = torch.zeros((1, 27, g.sizes()[1]), dtype=torch.float64, device="cuda")
    with pytest.raises(lt.LtError, match="ARG"):
        g.transfer(2, u, precision=1)
