"""The C ABI library loads, exports every symbol include/seraph.h declares,
and its host-side graph logic (in-edge CSR, equal-byte pages, argument
checks) works without a GPU through a host-only context."""
import os
import re
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sr():
    import paper_1806_00762_amd as sr
    if not os.path.exists(sr.LIB_PATH):
        from paper_1806_00762_amd import _build
        _build.build()
    sr.lib()
    return sr


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(sr_[a-z0-9_]+)\s*\(", txt))
    return names


def test_exports_every_declared_symbol(sr):
    out = subprocess.run(["nm", "-D", "--defined-only", sr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (sr_[a-z0-9_]+)", out))
    declared = declared_functions()
    assert declared, "no declarations found"
    missing = declared - exported
    assert not missing, f"declared but not exported: {sorted(missing)}"
    # the binding knows every declared function
    assert declared <= set(sr.exported_symbols())


def test_host_only_context_refuses_device_work(sr):
    c = sr.Context(-1, 1 << 30)
    g = c.load(graphgen.rmat(8, 4, seed=1, weights=(1, 9, 2)))
    with pytest.raises(sr.SeraphError) as e:
        g.run("sssp")
    assert e.value.status == sr.SR_EDEVICE
    g.close(); c.close()


def test_gather_probe_argument_checks(sr):
    """The probe checks its arguments before touching a device, and a
    host-only context has none to probe."""
    import numpy as np
    c = sr.Context(-1, 1 << 30)
    w = np.arange(16, dtype=np.uint32)
    v = np.arange(4, dtype=np.uint32)
    for words, vals, reps in ((w[:0], v, 1), (w, v[:0], 1), (w, v, 0)):
        with pytest.raises(sr.SeraphError) as e:
            sr.probe_gather(c, words, 0xFFFFFFFF, vals, repeats=reps)
        assert e.value.status == sr.SR_EINVAL
    with pytest.raises(sr.SeraphError) as e:
        sr.probe_gather(c, w, 0xFFFFFFFF, v)
    assert e.value.status == sr.SR_EDEVICE
    c.close()


@pytest.mark.parametrize("sym", [False, True])
def test_in_csr_and_pages(sr, sym):
    c = sr.Context(-1, 1 << 30)
    src = graphgen.rmat(11, 8, seed=5, weights=(1, 255, 3))
    G = c.load(src, symmetrize=sym)
    A = sp.csr_matrix((src.weights.astype(np.int64), src.col, src.offsets), shape=(src.n, src.n))
    if sym:
        A = A.maximum(A.T) if False else A
        # min weight over both directions, union of arcs
        B = A.T.tocsr()
        Ad = A.toarray(); Bd = B.toarray()
        both = (Ad > 0) & (Bd > 0)
        M = np.where(both, np.minimum(Ad, Bd), Ad + Bd)
        np.fill_diagonal(M, 0)
        IN = sp.csr_matrix(M.T)
    else:
        IN = A.T.tocsr()
    IN.sort_indices()
    for parts in (1, 3, 7):
        G.partition(parts, 4)
        info = G.info()
        assert info["m"] == IN.nnz
        offs, srcs, ws, vb = [0], [], [], 0
        for p in range(info["num_parts"]):
            pg = G.page(p)
            assert pg["v_begin"] == vb
            vb = pg["v_end"]
            offs.extend((pg["offsets"][1:] + offs[-1]).tolist())
            srcs.append(pg["src"]); ws.append(pg["weights"])
            # equal-byte split: a page's streamed bytes (4 per vertex, 4 per
            # edge word, 4 more per edge for separate weights) exceed
            # total/parts by at most one vertex's bytes
            eb = 8 if (pg["weights"] is not None and not pg["src_packed"]) else 4
            maxcost = 4 + eb * int(np.diff(IN.indptr).max())
            total = 4 * src.n + eb * IN.nnz
            cost = 4 * (pg["v_end"] - pg["v_begin"]) + eb * int(pg["offsets"][-1])
            assert cost <= -(-total // parts) + maxcost
        assert vb == src.n
        assert np.array_equal(np.array(offs), IN.indptr)
        assert np.array_equal(np.concatenate(srcs), IN.indices)
        assert np.array_equal(np.concatenate(ws), IN.data.astype(np.uint32))
    G.close(); c.close()


@pytest.mark.parametrize("parts", [1, 2, 4, 7, 64])
def test_equal_edge_pages(sr, parts):
    """SR_PART_EQUAL_EDGES: boundary i is the first vertex whose in-edges
    start at or after ceil(i * m / parts), empty ranges dropped (a vertex
    never straddles two pages). The expected cut is computed here from the
    in-degree counts of the input, not read back from the library."""
    c = sr.Context(-1, 1 << 30)
    src = graphgen.recipes.pagerank_s16() if parts == 4 else graphgen.rmat(12, 8, seed=11)
    G = c.load(src)
    G.partition(parts, 4, equal_edges=True)
    indeg = np.bincount(src.col, minlength=src.n).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(indeg)])          # in-edges before each vertex
    m = int(start[-1])
    want = [0]
    for i in range(1, parts):
        b = int(np.searchsorted(start, -(-i * m // parts), side="left"))
        if want[-1] < b < src.n:
            want.append(b)
    want.append(src.n)
    info = G.info()
    got = [G.page(p)["v_begin"] for p in range(info["num_parts"])] + [src.n]
    assert got == want
    for p in range(info["num_parts"]):
        pg = G.page(p)
        # each page holds at most a share plus one vertex's in-edges
        assert int(pg["offsets"][-1]) <= -(-m // parts) + int(indeg.max())
    G.close(); c.close()


def test_argument_checks(sr):
    c = sr.Context(-1, 1 << 30)
    bad = graphgen.Graph(3, np.array([0, 1, 2, 2]), np.array([1, 5], dtype=np.int32), None)
    with pytest.raises(sr.SeraphError) as e:
        c.load(bad)
    assert e.value.status == sr.SR_EINVAL
    bad = graphgen.Graph(3, np.array([0, 2, 1, 2]), np.array([1, 2], dtype=np.int32), None)
    with pytest.raises(sr.SeraphError):
        c.load(bad)
    g = c.load(graphgen.rmat(6, 4, seed=1))
    with pytest.raises(sr.SeraphError):
        g.partition(-1, 4)
    with pytest.raises(sr.SeraphError):
        g.partition(2, 1)
    g.close(); c.close()


def test_default_diagram_matches_reading(sr):
    import oracle
    d = sr.default_diagram()
    ns, init, mask, succ, fail = oracle.weak_default_diagram()
    assert d.num_states == ns and d.initial_state == init and d.attempt_mask == mask
    assert list(d.on_success) == succ and list(d.on_fail) == fail


def test_symmetric_flag_verifies(sr):
    c = sr.Context(-1, 1 << 30)
    sym = graphgen.rmat(10, 8, seed=7, symmetrize=True)
    G = c.load(sym, symmetric=True)
    assert G.info()["symmetric"] == 1
    G.close()
    with pytest.raises(sr.SeraphError) as e:
        c.load(graphgen.rmat(10, 8, seed=7), symmetric=True)
    assert e.value.status == sr.SR_EINVAL
    c.close()


def test_wide_weights_kept_as_u32(sr):
    """Weights >= 256 keep a separate u32 section; below 256 they are packed
    into the top byte of the edge word (both lossless)."""
    c = sr.Context(-1, 1 << 30)
    for hi, packed in ((255, True), (70000, False)):
        src = graphgen.rmat(9, 8, seed=2, weights=(1, hi, 3))
        G = c.load(src)
        G.partition(2, 4)
        pages = [G.page(p) for p in range(G.info()["num_parts"])]
        ws = np.concatenate([pg["weights"] for pg in pages])
        srcs = np.concatenate([pg["src"] for pg in pages])
        assert all(pg["src_packed"] == packed for pg in pages)
        A = sp.csr_matrix((src.weights.astype(np.int64), src.col, src.offsets), shape=(src.n, src.n)).T.tocsr()
        A.sort_indices()
        assert np.array_equal(ws, A.data.astype(np.uint32))
        assert np.array_equal(srcs, A.indices)
        # a packed page streams 4 bytes per weighted edge, an unpacked one 8
        m_p = sum(len(pg["src"]) for pg in pages)
        stream = sum(pg["stream_bytes"] for pg in pages)
        assert (stream < 8 * m_p) == packed
        G.close()
    c.close()


def test_packing_needs_24_bit_ids(sr):
    """Above 2^24 vertices the source id needs the top byte: weights stay separate."""
    c = sr.Context(-1, 1 << 31)
    n = (1 << 24) + 2
    g = graphgen.from_edges(n, [0, n - 1, 5], [n - 1, 3, 0], [7, 9, 11])
    G = c.load(g)
    G.partition(1, 2)
    pg = G.page(0)
    assert not pg["src_packed"]
    assert sorted(pg["src"].tolist()) == [0, 5, n - 1]
    assert sorted(pg["weights"].tolist()) == [7, 9, 11]
    G.close()
    c.close()


@pytest.mark.parametrize("symmetrize", [False, True])
def test_reorder_relabels_by_degree(sr, symmetrize):
    """SR_LOAD_REORDER: internal ids by descending in-degree (total degree
    when symmetrized), ties by the caller's id; the pages are the in-edge CSR
    of the relabeled graph."""
    src = graphgen.rmat(10, 8, seed=21, weights=(1, 255, 22))
    c = sr.Context(-1, 1 << 30)
    G = c.load(src, symmetrize=symmetrize, reorder=True)
    internal_of, caller_of = G.order()
    n = src.n
    assert np.array_equal(np.sort(internal_of), np.arange(n))
    assert np.array_equal(caller_of[internal_of], np.arange(n))
    A = sp.csr_matrix((src.weights.astype(np.int64), src.col, src.offsets), shape=(n, n))
    deg = np.asarray((A != 0).sum(axis=0)).ravel()          # in-degree
    if symmetrize:
        deg = deg + np.diff(src.offsets)
    key = np.lexsort((np.arange(n), -deg))                  # descending degree, then id
    assert np.array_equal(caller_of, key)
    # expected in-CSR of the relabeled graph
    P = sp.csr_matrix((np.ones(n), (internal_of, np.arange(n))), shape=(n, n))
    B = (P @ A @ P.T).tocsr()
    G.partition(3, 4)
    offs, srcs, vb = [0], [], 0
    for p in range(G.info()["num_parts"]):
        pg = G.page(p)
        assert pg["v_begin"] == vb
        vb = pg["v_end"]
        offs.extend((pg["offsets"][1:] + offs[-1]).tolist())
        srcs.append(pg["src"])
    if not symmetrize:
        IN = B.T.tocsr()
        IN.sort_indices()
        assert np.array_equal(np.array(offs), IN.indptr)
        assert np.array_equal(np.concatenate(srcs), IN.indices)
    else:
        # undirected: row v lists the internal ids adjacent to v
        U = sp.csr_matrix((np.ones(src.m), (internal_of[np.repeat(np.arange(n), np.diff(src.offsets))],
                                            internal_of[src.col])), shape=(n, n))
        U = ((U + U.T) > 0).astype(np.int8).tocsr()
        U.setdiag(0)
        U.eliminate_zeros()
        U.sort_indices()
        assert np.array_equal(np.array(offs), U.indptr)
        assert np.array_equal(np.concatenate(srcs), U.indices)
    assert G.info()["reordered"] == 1
    G.close()
    H = c.load(src)
    with pytest.raises(sr.SeraphError) as e:
        H.order()
    assert e.value.status == sr.SR_ESTATE
    H.close()
    c.close()
