"""Pins of the oracle's neighbour infrastructure (Sec. 3.4 and the reference-configuration
neighbour sets of Sec. 2.2) against an O(N^2) brute force and the paper's worked example."""
import numpy as np
import pytest

import oracle
import workloads


def brute_topology(X, dp, h_over_dp=1.3):
    """Cells of size r_c = 2h from the bounding-box minimum, stable order by (cell, input index),
    rows = every other particle with squared distance below r_c^2, ascending internal index."""
    n, D = X.shape
    h = h_over_dp * dp
    rc = 2.0 * h
    rc2 = rc * rc
    xmin = X.min(axis=0)
    cxyz = np.floor((X - xmin[None, :]) / rc).astype(np.int64)
    nc = cxyz.max(axis=0) + 1
    if D == 2:
        lin = cxyz[:, 0] * nc[1] + cxyz[:, 1]
    else:
        lin = (cxyz[:, 0] * nc[1] + cxyz[:, 1]) * nc[2] + cxyz[:, 2]
    perm = np.argsort(lin, kind="stable")
    Xs = X[perm]
    d = Xs[None, :, :] - Xs[:, None, :]
    r2 = d[:, :, 0] * d[:, :, 0] + d[:, :, 1] * d[:, :, 1]
    if D == 3:
        r2 = r2 + d[:, :, 2] * d[:, :, 2]
    adj = r2 < rc2
    np.fill_diagonal(adj, False)
    row_ptr = np.concatenate([[0], np.cumsum(adj.sum(axis=1))])
    col = np.nonzero(adj)[1]
    cx = cxyz[perm]
    if D == 2:
        colour = 3 * (cx[:, 0] % 3) + (cx[:, 1] % 3)
    else:
        colour = 9 * (cx[:, 0] % 3) + 3 * (cx[:, 1] % 3) + (cx[:, 2] % 3)
    return dict(perm=perm, cell=lin[perm], colour=colour, row_ptr=row_ptr, col=col, cxyz=cx, nc=nc)


CASES = [
    (2, (12, 5), 2, 0.0),
    (2, (17, 6), 3, 0.1),
    (3, (7, 4, 5), 2, 0.0),
    (3, (9, 5, 4), 2, 0.1),
    (3, (6, 6, 6), 1, 0.3),
]


@pytest.mark.parametrize("dim,shape,nclamp,jitter", CASES)
def test_topology_matches_brute_force(dim, shape, nclamp, jitter):
    body = workloads.small_body(dim, shape, nclamp=nclamp, jitter=jitter, jitter_seed=dim)
    ob = oracle.OracleBody(body)
    got = ob.topology()
    ref = brute_topology(body.X0, body.dp)
    for k in ("perm", "cell", "colour", "row_ptr", "col"):
        assert np.array_equal(got[k], ref[k]), k
    # rows ascending, symmetric adjacency, every edge between cells at most one apart per axis
    rp, col = got["row_ptr"], got["col"]
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(np.diff(col)[np.diff(rows) == 0] > 0)
    pairs = set(zip(rows.tolist(), col.tolist()))
    assert all((j, i) in pairs for i, j in pairs)
    cx = ref["cxyz"]
    assert np.abs(cx[rows] - cx[col]).max() <= 1


@pytest.mark.parametrize("dim,shape,nclamp,jitter", CASES)
def test_same_colour_cells_have_disjoint_neighbourhoods(dim, shape, nclamp, jitter):
    """Sec. 3.4: cells of one block are never adjacent, so the particles that two cells of one
    colour touch (their own and their neighbours') are disjoint -- the race-freedom property."""
    body = workloads.small_body(dim, shape, nclamp=nclamp, jitter=jitter, jitter_seed=dim)
    t = oracle.OracleBody(body).topology()
    rp, col, cell, colour = t["row_ptr"], t["col"], t["cell"], t["colour"]
    touched = {}
    for i in range(len(cell)):
        s = touched.setdefault(int(cell[i]), set())
        s.add(i)
        s.update(col[rp[i]:rp[i + 1]].tolist())
    by_colour = {}
    for c, parts in touched.items():
        k = int(colour[np.nonzero(cell == c)[0][0]])
        by_colour.setdefault(k, []).append(parts)
    for k, sets in by_colour.items():
        seen = set()
        for s in sets:
            assert not (seen & s), f"colour {k} cells share particles"
            seen |= s


def test_colour_blocks_reproduce_paper_example(golden):
    """Sec. 3.4 sketch: on a 6 x 9 grid numbered from 1 (y fastest), block 1 = {1,4,7,28,31,34}
    and block 9 = {21,24,27,48,51,54}; colours run 0..8 for blocks 1..9."""
    g = golden["splitting_cll_blocks"]
    dp = 0.002
    # a lattice whose cell grid (cell = 2.6 dp) is exactly 6 x 9
    body = workloads.cantilever(2, (15, 23), dp, nclamp=0)
    ob = oracle.OracleBody(body)
    nc, _, _ = ob.grid()
    assert tuple(nc[:2]) == tuple(g["grid"])
    ncell = g["grid"][0] * g["grid"][1]
    blocks = {}
    for lin in range(ncell):
        blocks.setdefault(ob.cell_colour(lin), []).append(lin + 1)
    assert blocks[0] == g["block_1"]
    assert blocks[8] == g["block_9"]
    assert sorted(blocks) == list(range(9))
    assert all(len(v) == 6 for v in blocks.values())


def test_interior_neighbour_counts():
    """Support 2h = 2.6 dp on a square / cubic lattice holds 20 (2D) and 80 (3D) neighbours."""
    for dim, shape in ((2, (12, 12)), (3, (8, 8, 8))):
        body = workloads.small_body(dim, shape, nclamp=0)
        t = oracle.OracleBody(body).topology()
        counts = np.diff(t["row_ptr"])
        assert counts.max() == (20 if dim == 2 else 80)
