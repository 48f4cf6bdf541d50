"""Oracle pins for adaptation (Section 4.1) and strong 2:1 balance (Section 3.2).

The balanced tree is the unique coarsest refinement in which touching leaves
differ by at most one level.  It is pinned here by an independent brute force
on the finest-cell grid that splits one violating leaf at a time in random
order: any order must give the same tree."""
import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth

import brute

CASES = [(2, 4, 0), (2, 4, 1), (2, 4, 2), (2, 5, 2), (3, 3, 0), (3, 3, 1), (3, 3, 2)]


def _unbalanced_tree(dim, dmax, kind, seed):
    """Random adapts without balance, so 2:1 violations accumulate."""
    t = oracle.Tree(dim, 1, dmax, balance=kind)
    for c in range(dmax + 1):
        t.adapt(synth.random_flags(seed * 97 + c, t.size(), 0.3, 0.2))
    return t


@pytest.mark.parametrize("dim,dmax,kind", CASES)
def test_balance_matches_bruteforce(dim, dmax, kind):
    for seed in range(3):
        t = _unbalanced_tree(dim, dmax, kind, seed)
        before = t.keys()
        ref = brute.balance(dim, dmax, brute.leaves_of(dim, dmax, before), kind, seed=seed)
        ref_keys = brute.keys_of(dim, dmax, ref)
        t.balance(brute=False)
        assert np.array_equal(t.keys(), ref_keys)
        assert t.is_balanced()
        t2 = oracle.Tree(dim, 1, dmax, balance=kind, keys=before)
        t2.balance(brute=True)
        assert np.array_equal(t2.keys(), ref_keys)
        # idempotent
        t.balance()
        assert np.array_equal(t.keys(), ref_keys)


@pytest.mark.parametrize("dim,dmax,kind", [(2, 5, 2), (3, 3, 2), (2, 5, 0)])
def test_balance_is_coarsest_locally(dim, dmax, kind):
    """Merging any family created by balance breaks 2:1 again."""
    t = _unbalanced_tree(dim, dmax, kind, 11)
    before = set(int(k) for k in t.keys())
    pre = brute.leaves_of(dim, dmax, t.keys())
    t.balance()
    after = brute.leaves_of(dim, dmax, t.keys())
    pre_internal_or_leaf = set()
    for d, a in pre:
        # every ancestor-or-self of an input leaf is "not created by balance"
        for dd in range(d + 1):
            s = 1 << (dmax - dd)
            pre_internal_or_leaf.add((dd, tuple(x - x % s for x in a)))
    fams = {}
    for i, (d, a) in enumerate(after):
        if d == 0:
            continue
        s = 1 << (dmax - d + 1)
        fams.setdefault((d - 1, tuple(x - x % s for x in a)), []).append(i)
    checked = 0
    for parent, kids in fams.items():
        if len(kids) != (1 << dim):
            continue
        # families whose parent was internal in the input are not balance's doing
        d, a = parent
        internal_before = any(dd > d and all(aa - aa % (1 << (dmax - d)) == pa for aa, pa in zip(aa_, a))
                              for dd, aa_ in pre)
        if internal_before:
            continue
        merged = [lf for j, lf in enumerate(after) if j not in kids] + [parent]
        assert brute.violators(dim, dmax, merged, kind), f"family {parent} was not needed"
        checked += 1
    assert checked > 0
    assert before  # keep the input alive for debugging


@pytest.mark.parametrize("dim,dmax", [(2, 5), (3, 4)])
def test_adapt_semantics(dim, dmax):
    """Refine +1 once, coarsen only complete all -1 families, clamp at D_min/D_max."""
    t = oracle.Tree(dim, 2, dmax)
    for c in range(4):
        t.adapt(synth.random_flags(500 + c, t.size(), 0.3, 0.2))
        t.balance()
    for seed in range(3):
        old = brute.leaves_of(dim, dmax, t.keys())
        flags = synth.random_flags(900 + seed, len(old), 0.2, 0.6)
        t.adapt(flags)
        new = set(brute.leaves_of(dim, dmax, t.keys()))
        exp = set()
        fam = {}
        for (d, a), f in zip(old, flags):
            if d > 0:
                s = 1 << (dmax - d + 1)
                fam.setdefault((d - 1, tuple(x - x % s for x in a)), []).append((d, a, int(f)))
        gone = set()
        for parent, kids in fam.items():
            if len(kids) == (1 << dim) and all(k[2] == -1 for k in kids) and parent[0] >= 2:
                exp.add(parent)
                gone.update((k[0], k[1]) for k in kids)
        for (d, a), f in zip(old, flags):
            if (d, a) in gone:
                continue
            if f == 1 and d < dmax:
                exp.update(brute.split(dim, dmax, (d, a)))
            else:
                exp.add((d, a))
        assert new == exp
        t.balance()


def test_adapt_rejects_bad_flags():
    t = oracle.Tree(2, 2, 5)
    f = np.zeros(t.size(), dtype=np.int8)
    f[3] = 2
    with pytest.raises(oracle.OracleError):
        t.adapt(f)


@pytest.mark.parametrize("dim,dmax", [(2, 6), (3, 4)])
def test_mapping_uses_every_old_leaf_once(dim, dmax):
    """Every new leaf is an old leaf, a child of one, or the parent of 2^dim
    old leaves (each old leaf used exactly once) after adapt + balance."""
    t = oracle.Tree(dim, 2, dmax)
    for c in range(5):
        t.adapt(synth.random_flags(70 + c, t.size(), 0.3, 0.4))
        t.balance()
        src, kind = t.map()
        used = np.zeros(t.old_size(), dtype=np.int64)
        for s, k in zip(src, kind):
            if k == 0:
                used[s] += 1
            elif k == -1:
                used[s:s + (1 << dim)] += 1
        # refined children share one parent: count each parent once
        par = set(int(s) for s, k in zip(src, kind) if k > 0)
        for s in par:
            used[s] += 1
        assert (used == 1).all()
        assert set(int(k) for k in kind if k > 0) <= set(range(1, (1 << dim) + 1))
