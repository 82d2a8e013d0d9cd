"""The named synthetic workloads against their recipes (stand-ins for the
paper's CI Hamiltonians, Table 2, at the sizes of its experiments, Section 5).

Each expected value below follows from the recipe in `synth/workloads.py`
by counting, not from a run of the generator: a wrong stream, a dropped
symmetrisation or a mis-scaled draw moves one of them by many standard
errors.  The tiled recipe is checked at n = 256,000 (4,000 tile-rows), where
its per-tile and per-row statistics are those of the full-size matrix.
"""
import numpy as np

from synth import workloads as W


def _strict_upper(A):
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = A.col > rows
    return rows[off], A.col[off], A.val[off]


def test_random_sym_20k_recipe():
    """n = 20,000, FP64; d = sort(U[0, 200)); each row draws 50 distinct
    partners among the other n - 1 rows, value N(0,1) * 0.5, summed into the
    symmetric pair.  A pair is drawn from both ends with probability
    (50 / (n - 1))^2, so a full row holds 2 * 50 - 50^2 / (n - 1) = 99.875
    off-diagonal entries on average, and the stored triangle about
    n * 99.875 / 2 = 998,750 of them."""
    A = W.make_matrix("random_sym_20k")
    assert A.n == 20000 and A.val.dtype == np.float64
    r, c, v = _strict_upper(A)
    expect = 2 * 50 - 50 ** 2 / (A.n - 1)
    assert abs(2 * r.size / A.n - expect) < 0.05
    assert abs(r.size - A.n * expect / 2) < 1000
    # values: N(0,1) * 0.5 (pairs drawn twice, 0.125% of them, add variance 0.25)
    assert abs(v.std() - 0.5) < 3e-3 and abs(v.mean()) < 3e-3
    d = np.asarray(A.diag)
    assert np.all(np.diff(d) >= 0) and d[0] >= 0 and d[-1] < 200
    # order statistics of 20,000 uniforms: the extremes sit within ~0.01 * 200 / 20 of the ends
    assert d[0] < 0.1 and d[-1] > 199.9
    # the partners are uniform over the columns: each tenth of the column range
    # holds a tenth of the off-diagonal entries (both triangles counted)
    cols = np.concatenate([r, c])
    frac = np.bincount(cols * 10 // A.n, minlength=10) / cols.size
    assert np.all(np.abs(frac - 0.1) < 0.003)


def test_tiled_recipe():
    """64 x 64 tiles; each tile-row draws 47 distinct tile columns among the
    other T - 1, and the tile pattern is symmetrised, so a tile-row meets
    (T - 1) (2q - q^2) = 94 - 47^2 / (T - 1) off-diagonal tiles (q = 47 / (T - 1));
    each entry of a present tile is kept with p = 400 / (64 * 95), so an
    off-diagonal tile holds 4096 p = 269.47 entries on average and a full row
    about 64 p * 94 = 395.8 off-diagonal entries; values N(0,1) * 0.1, FP32;
    d = sort(U[0, 500))."""
    T = 4000
    A = W.make_matrix("tiled_2m", n=64 * T)
    assert A.val.dtype == np.float32
    r, c, v = _strict_upper(A)
    ti, tj = r // 64, c // 64
    od = ti != tj
    key = ti[od].astype(np.int64) * T + tj[od]
    tiles, per_tile = np.unique(key, return_counts=True)
    p = 400.0 / (64 * 95)
    # entries per off-diagonal tile: Binomial(4096, p), sd 16, averaged over ~187,000 tiles
    assert abs(per_tile.mean() - 4096 * p) < 0.3
    assert abs(per_tile.std() - np.sqrt(4096 * p * (1 - p))) < 0.5
    # off-diagonal tiles per full tile-row
    per_row = np.bincount(tiles // T, minlength=T) + np.bincount(tiles % T, minlength=T)
    assert abs(per_row.mean() - (94 - 47 ** 2 / (T - 1))) < 0.3
    # full off-diagonal entries per row: the off-diagonal tiles' share plus the
    # diagonal tile's (63 other columns in the tile, each kept with p)
    full = 2 * r.size / A.n
    assert abs(full - (64 * p * (94 - 47 ** 2 / (T - 1)) + 63 * p)) < 1.0
    assert abs(float(v.std()) - 0.1) < 1e-3 and abs(float(v.mean())) < 1e-3
    d = np.asarray(A.diag)
    assert np.all(np.diff(d) >= 0) and d[0] >= 0 and d[-1] < 500


def test_recipes_are_deterministic_per_seed():
    """The generator is counter-based: a seed gives the same matrix on every
    call, another seed a different one."""
    a = W.make_matrix("random_sym_1k", seed=5)
    b = W.make_matrix("random_sym_1k", seed=5)
    c = W.make_matrix("random_sym_1k", seed=6)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert np.array_equal(a.val, b.val) and np.array_equal(a.diag, b.diag)
    assert not (a.col.size == c.col.size and np.array_equal(a.col, c.col))
