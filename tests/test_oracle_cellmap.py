"""Pins of the oracle's cell map (paper Sec. 6.2.1, read in the 0-based floor
form with clamping): literal cell indices computed by hand, the linear cell
order, entry / box / slot counts of a tiny mesh counted by hand, and the
monotonicity that the home-cell rule rests on.

Each case is chosen so that one plausible mistake fails it:
  * the paper's 1-based ceiling index, shifted to 0-based (ceil(t) - 1),
    puts a coordinate on a cell edge into the lower cell;
  * a clamp to n instead of n - 1 gives an index past the grid;
  * a different linearisation order gives other strides per axis.
"""
import numpy as np
import pytest

import oracle
import synth


# ------------------------------------------------------------------ cell_of

@pytest.mark.parametrize("x,wlo,inv,n,want", [
    (0.5, 0.0, 4.0, 10, 2),       # t = 2.0 exactly: on an edge, the upper cell (ceil - 1 gives 1)
    (0.4999999999, 0.0, 4.0, 10, 1),
    (0.6, 0.0, 4.0, 10, 2),       # t = 2.4
    (0.0, 0.0, 4.0, 10, 0),       # the world origin is cell 0 (ceil - 1 gives -1)
    (1.0, 1.0, 3.0, 5, 0),
    (2.0, 1.0, 3.0, 5, 3),        # t = 3.0, edge
    (-7.25, -8.0, 2.0, 5, 1),     # t = 1.5
    (-9.0, -8.0, 2.0, 5, 0),      # below the world: clamps to 0
    (1.0e9, 0.0, 1.0, 5, 4),      # above the last cell: clamps to n - 1 (not n)
    (5.0, 0.0, 1.0, 5, 4),        # t = n exactly: n - 1
    (4.999, 0.0, 1.0, 5, 4),
    (3.0, 0.0, 1.0, 1, 0),        # a single cell holds everything
    (float("nan"), 0.0, 1.0, 5, 0),
    (float("inf"), 0.0, 1.0, 5, 4),
    (float("-inf"), 0.0, 1.0, 5, 0),
])
def test_cell_of_literal(x, wlo, inv, n, want):
    assert oracle.cell_of(x, wlo, inv, n) == want


def test_cell_of_rounds_the_product_once():
    """t = (x - w_lo) * inv in FP64, each operation rounded once: with
    x - w_lo = 0.3 (inexact) and inv = 10, the product rounds to 3.0 exactly
    (0.3 is stored as 0.29999999999999998889...; times 10 rounds to 3.0), so
    the coordinate lies in cell 3; an evaluation in higher precision would
    give 2."""
    d = 0.3
    assert d * 10.0 == 3.0
    assert oracle.cell_of(d, 0.0, 10.0, 100) == 3


# -------------------------------------------------------- linear cell order

def _one_quad(W00, W10, W01, W11):
    """A non-periodic 2 x 2 vertex grid: one quad, triangles T1 (t = 0) and
    T2 (t = 1).  verts[k][i] = W(i, k)."""
    V = np.zeros((2, 2, 4))
    V[0, 0], V[0, 1], V[1, 0], V[1, 1] = W00, W10, W01, W11
    return synth.Mesh(V, np.array([0.0, 1.0]), np.array([0.0, 1.0]), False)


N_CELLS = np.array([3, 4, 5, 6], np.int64)      # distinct per axis: each axis has its own stride
W_LO = np.zeros(4)


@pytest.mark.parametrize("axis,stride", [(0, 4 * 5 * 6), (1, 5 * 6), (2, 6), (3, 1)])
def test_linear_order_per_axis(axis, stride):
    """A triangle inside cell 1 along one axis and cell 0 along the others
    has the single linear id ((c0 n1 + c1) n2 + c2) n3 + c3 = the stride of
    that axis: 120, 30, 6, 1 for n = (3, 4, 5, 6)."""
    base = np.full(4, 0.25)
    p = base.copy()
    p[axis] = 1.25
    q = p.copy()
    q[(axis + 1) % 4] += 0.5
    r = p.copy()
    r[(axis + 2) % 4] += 0.5
    m = _one_quad(q, p, r, r)            # T1 = (W(1,0), W(0,0), W(0,1)) = (p, q, r)
    cells = oracle.tri_entries(m, 0, W_LO, 1.0, N_CELLS)
    assert cells.tolist() == [stride]


# ------------------------------------------------------ a mesh counted by hand

# W(0,0), W(1,0), W(0,1), W(1,1) with edge 1 and n = (3, 4, 5, 6):
#   T1 = (W(1,0), W(0,0), W(0,1)): x in [0.5, 1.0] -> cells 0..1 (1.0 is an edge: upper cell),
#        y in [0.5, 2.5] -> 0..2, z = w = 0.5 -> 0: 2 * 3 * 1 * 1 = 6 cells,
#        linear ids (c0 * 4 + c1) * 30 = 0, 30, 60, 120, 150, 180;
#   T2 = (W(0,1), W(1,1), W(1,0)): x in [0.5, 1.5] -> 0..1, y in [0.5, 2.5] -> 0..2,
#        z in [0.5, 7.0] -> 0..4 (7 clamps to n - 1 = 4), w in [-3.0, 0.5] -> 0 (clamped):
#        2 * 3 * 5 * 1 = 30 cells.
HAND = dict(W00=(0.5, 0.5, 0.5, 0.5), W10=(1.0, 0.5, 0.5, 0.5), W01=(0.5, 2.5, 0.5, 0.5),
            W11=(1.5, 2.5, 7.0, -3.0))


def _hand_mesh():
    return _one_quad(*(np.array(HAND[k]) for k in ("W00", "W10", "W01", "W11")))


def test_hand_mesh_entries():
    m = _hand_mesh()
    assert oracle.tri_entries(m, 0, W_LO, 1.0, N_CELLS).tolist() == [0, 30, 60, 120, 150, 180]
    t2 = oracle.tri_entries(m, 1, W_LO, 1.0, N_CELLS)
    want = sorted(((c0 * 4 + c1) * 5 + c2) * 6 for c0 in range(2) for c1 in range(3) for c2 in range(5))
    assert len(t2) == 30 and t2.tolist() == want        # emitted in lexicographic order
    assert oracle.grid_entries(m, W_LO, 1.0, N_CELLS) == 36


def test_hand_mesh_boxes_and_slots():
    """The mesh against itself: T1's 6 cells hold 2 A and 2 B entries (4
    slots each), the other 24 cells of T2 hold 1 and 1: 30 boxes, 6 * 4 + 24
    = 48 slots, 72 entries.  Candidates: all 4 pairs (the boxes overlap)."""
    m = _hand_mesh()
    g = oracle.grid_search(m, m, W_LO, 1.0, N_CELLS)
    assert g.n_entries == 72
    assert g.n_boxes == 30
    assert g.n_slots == 48
    assert g.cand.tolist() == [(0 << 32) | 0, (0 << 32) | 1, (1 << 32) | 0, (1 << 32) | 1]


def test_hand_mesh_nonfinite_has_no_entries():
    m = _hand_mesh()
    m.verts = m.verts.copy()
    m.verts[1, 1, 3] = np.nan            # W(1,1) belongs to T2 only
    assert oracle.tri_entries(m, 1, W_LO, 1.0, N_CELLS) is None
    assert oracle.grid_entries(m, W_LO, 1.0, N_CELLS) == 6


# ------------------------------------------------------------- monotonicity

def test_cell_of_is_monotone():
    """x1 <= x2 implies cell(x1) <= cell(x2), for random grids and for
    coordinates on and next to cell edges (the property that puts the home
    cell of an overlapping pair inside both cell ranges)."""
    rng = np.random.default_rng(7)
    for _ in range(40):
        wlo = rng.uniform(-3, 3)
        inv = float(np.exp(rng.uniform(-3, 3)))
        n = int(rng.integers(1, 50))
        edges = wlo + np.arange(-2, n + 3) / inv
        xs = np.concatenate([rng.uniform(wlo - 3 / inv, wlo + (n + 3) / inv, 200), edges,
                             np.nextafter(edges, -np.inf), np.nextafter(edges, np.inf)])
        xs.sort()
        cs = [oracle.cell_of(x, wlo, inv, n) for x in xs]
        assert all(0 <= c < n for c in cs)
        assert all(a <= b for a, b in zip(cs, cs[1:]))


def test_home_cell_lies_in_both_ranges():
    """For random overlapping boxes the cell of the componentwise max of the
    lower corners lies in both boxes' cell ranges, per axis."""
    rng = np.random.default_rng(8)
    for _ in range(2000):
        wlo, inv, n = rng.uniform(-1, 1), float(np.exp(rng.uniform(-1, 3))), int(rng.integers(1, 30))
        a = np.sort(rng.uniform(-2, 2, 2))
        b = np.sort(rng.uniform(-2, 2, 2))
        if a[0] > b[1] or b[0] > a[1]:
            continue
        h = oracle.cell_of(max(a[0], b[0]), wlo, inv, n)
        for lo, hi in (a, b):
            assert oracle.cell_of(lo, wlo, inv, n) <= h <= oracle.cell_of(hi, wlo, inv, n)
