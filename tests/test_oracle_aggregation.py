"""Pins of the oracle's MIS-2 aggregation (distance-2 maximal independent set)."""
import numpy as np
import pytest
import scipy.sparse as sp

from amgf_inputs import make_config
from oracle import fmix32, mis2_sequential, aggregate, strength_graph
from oracle.amgf_oracle import priority_keys
from oracle_util import build


def _fmix32_int(h):
    M = 0xFFFFFFFF
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & M
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & M
    h ^= h >> 16
    return h


def test_fmix32_is_the_murmur3_finalizer_and_bijective():
    a = np.arange(1 << 20, dtype=np.uint32)
    h = fmix32(a)
    assert len(np.unique(h)) == len(a)
    for v in [0, 1, 2, 12345, 0xFFFFFFFF, 0x80000000]:
        assert int(fmix32(np.uint32(v))) == _fmix32_int(v)
    assert int(fmix32(np.uint32(0))) == 0


def _random_graph(n, deg, seed):
    rng = np.random.default_rng(seed)
    r = rng.integers(0, n, n * deg)
    c = rng.integers(0, n, n * deg)
    keep = r != c
    G = sp.coo_matrix((np.ones(keep.sum()), (r[keep], c[keep])), shape=(n, n))
    G = ((G + G.T) > 0).astype(np.int64).tocsr()
    G.sort_indices()
    return G.indptr.astype(np.int64), G.indices.astype(np.int64)


def _dist2(rp, col):
    n = len(rp) - 1
    G = sp.csr_matrix((np.ones(len(col)), col, rp), shape=(n, n))
    I = sp.identity(n, format="csr")
    return (((I + G) @ (I + G)) > 0).tocsr()


def _lexfirst_characterisation(rp, col, active, root):
    """Independent characterisation of the greedy (lexicographically first) MIS-2:
    roots are pairwise >= 3 apart, and every active non-root has a root of higher
    priority within distance 2."""
    n = len(rp) - 1
    key = priority_keys(n)
    D2 = _dist2(rp, col)
    for v in range(n):
        nb = D2.indices[D2.indptr[v]:D2.indptr[v + 1]]
        if root[v]:
            assert not root[nb[nb != v]].any()
        elif active[v]:
            rr = nb[root[nb]]
            assert len(rr) and key[rr].max() > key[v]
        else:
            assert not root[v]


def _parallel_rounds(rp, col, active):
    """Second algorithm: parallel rounds; a node joins when it carries the largest
    undecided key in its distance-2 ball; nodes near a root drop out."""
    n = len(rp) - 1
    key = priority_keys(n).astype(np.float64)   # exact: keys < 2^53 for n < 2^21
    key = priority_keys(n)
    rows = np.repeat(np.arange(n), np.diff(rp))
    UND, ROOT, OUT = 0, 1, 2
    st = np.where(active, UND, OUT)
    INF = np.uint64(0xFFFFFFFFFFFFFFFF)
    for _ in range(200):
        if not (st == UND).any():
            break
        code = np.where(st == ROOT, INF, np.where(st == UND, key, np.uint64(0)))
        m1 = code.copy()
        np.maximum.at(m1, rows, code[col])
        m2 = m1.copy()
        np.maximum.at(m2, rows, m1[col])
        und = st == UND
        st = np.where(und & (m2 == INF), OUT, np.where(und & (m2 == key), ROOT, st))
    return st == ROOT


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mis2_random_graphs(seed):
    rp, col = _random_graph(300, 2, seed)
    active = np.diff(rp) > 0
    root = mis2_sequential(rp, col, active)
    _lexfirst_characterisation(rp, col, active, root)
    assert (root == _parallel_rounds(rp, col, active)).all()


@pytest.fixture(scope="module")
def c1():
    p = make_config("C1")
    return p, build(p)


def test_mis2_and_aggregates_on_the_strength_graph(c1):
    p, o = c1
    lev = o.levels[0]
    rp, col, w = lev.G
    active = np.diff(rp) > 0
    _lexfirst_characterisation(rp, col, active, lev.roots)
    assert (lev.roots == _parallel_rounds(rp, col, active)).all()
    agg = lev.agg
    # partition of the active nodes, one root per aggregate, ids by ascending root
    assert ((agg >= 0) == active).all()
    rid = np.nonzero(lev.roots)[0]
    assert (agg[rid] == np.arange(len(rid))).all()
    assert len(np.unique(agg[agg >= 0])) == lev.n_agg == len(rid)
    rows = np.repeat(np.arange(len(agg)), np.diff(rp))
    # every root neighbour is in the root's aggregate; every member touches its aggregate
    for r in rid:
        assert (agg[col[rp[r]:rp[r + 1]]] == agg[r]).all()
    same = agg[rows] == agg[col]
    has = np.bincount(rows[same], minlength=len(agg)) > 0
    assert has[active].all()


def test_coarse_levels_aggregate_on_aggregate_adjacency():
    """Level l+1 graph: aggregates I ~ J iff a level-l edge joins a node of I to one of J."""
    p = make_config("C1")
    o = build(p, coarse_max_nodes=8)
    assert o.nlev >= 3
    l0, l1 = o.levels[0], o.levels[1]
    rp, col, _ = l0.G
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    ref = set()
    for a, b in zip(rows, col):
        I, J = l0.agg[a], l0.agg[b]
        if I >= 0 and J >= 0 and I != J:
            ref.add((int(I), int(J)))
    rp1, col1, _ = l1.G
    rows1 = np.repeat(np.arange(len(rp1) - 1), np.diff(rp1))
    got = set(zip(rows1.tolist(), col1.tolist()))
    assert got == ref
    # every coarse graph edge is also a block of the Galerkin operator
    assert (l1.A.find(rows1, col1) >= 0).all()
