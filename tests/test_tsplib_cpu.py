"""The TSPLIB reader against the format's published definitions: the
distance functions on hand-computed pairs, every EXPLICIT layout written out
by its own definition here, node order, round trips and rejections.  The
instances are synthetic (no TSPLIB instance is reproduced)."""
import numpy as np
import pytest

import aco_instances as inst
from aco_instances import tsplib as T


def _coord_text(coords, ewt="EUC_2D", order=None, sep=" : "):
    n = len(coords)
    order = range(n) if order is None else order
    lines = ["NAME%ssynthetic" % sep, "TYPE%sTSP" % sep, "DIMENSION%s%d" % (sep, n),
             "EDGE_WEIGHT_TYPE%s%s" % (sep, ewt), "NODE_COORD_SECTION"]
    lines += ["%d %r %r" % (i + 1, float(coords[i][0]), float(coords[i][1])) for i in order]
    return "\n".join(lines + ["EOF"]) + "\n"


def test_euc_2d_rounds_to_nearest_with_halves_up():
    # distances 3, 4, 5 (the 3-4-5 triangle), 1.5 -> 2 and 2.4 -> 2
    c = [(0.0, 0.0), (3.0, 0.0), (3.0, 4.0), (0.0, 1.5), (0.0, -2.4)]
    W = T.tsplib_weights(T.parse_tsplib(_coord_text(c)))
    assert (W[0, 1], W[1, 2], W[0, 2]) == (3, 4, 5)
    assert W[0, 3] == 2 and W[0, 4] == 2
    assert np.array_equal(W, W.T) and not W.diagonal().any()


def test_ceil_2d_rounds_up():
    c = [(0.0, 0.0), (1.0, 1.0), (3.0, 4.0), (0.0, 2.0)]
    W = T.tsplib_weights(T.parse_tsplib(_coord_text(c, "CEIL_2D")))
    assert W[0, 1] == 2          # sqrt 2
    assert W[0, 2] == 5          # exactly 5 stays 5
    assert W[0, 3] == 2


def test_att_pseudo_euclidean():
    # r = sqrt(d^2 / 10); t = nint(r); t + 1 when t < r
    c = [(0.0, 0.0), (10.0, 0.0), (30.0, 40.0), (0.0, 20.0)]
    W = T.tsplib_weights(T.parse_tsplib(_coord_text(c, "ATT")))
    assert W[0, 1] == 4   # r = sqrt(10) = 3.162..., t = 3 < r
    assert W[0, 2] == 16  # r = sqrt(250) = 15.81..., t = 16 >= r
    assert W[0, 3] == 7   # r = sqrt(40) = 6.324..., t = 6 < r


def _explicit_text(W, fmt):
    """EDGE_WEIGHT_SECTION of a symmetric W in layout `fmt`, written from the
    layout's definition (rows: row by row; cols: column by column)."""
    n = W.shape[0]
    vals = []
    if fmt == "FULL_MATRIX":
        vals = [W[i, j] for i in range(n) for j in range(n)]
    elif fmt == "UPPER_ROW":
        vals = [W[i, j] for i in range(n) for j in range(i + 1, n)]
    elif fmt == "LOWER_ROW":
        vals = [W[i, j] for i in range(n) for j in range(i)]
    elif fmt == "UPPER_DIAG_ROW":
        vals = [W[i, j] for i in range(n) for j in range(i, n)]
    elif fmt == "LOWER_DIAG_ROW":
        vals = [W[i, j] for i in range(n) for j in range(i + 1)]
    elif fmt == "UPPER_COL":      # column j, rows above the diagonal
        vals = [W[i, j] for j in range(n) for i in range(j)]
    elif fmt == "LOWER_COL":      # column j, rows below the diagonal
        vals = [W[i, j] for j in range(n) for i in range(j + 1, n)]
    elif fmt == "UPPER_DIAG_COL":
        vals = [W[i, j] for j in range(n) for i in range(j + 1)]
    elif fmt == "LOWER_DIAG_COL":
        vals = [W[i, j] for j in range(n) for i in range(j, n)]
    # a ragged line layout, as files use
    body = []
    for k in range(0, len(vals), 7):
        body.append(" ".join(str(int(v)) for v in vals[k:k + 7]))
    return "\n".join(["NAME: explicit", "TYPE: TSP", "DIMENSION: %d" % n,
                      "EDGE_WEIGHT_TYPE: EXPLICIT", "EDGE_WEIGHT_FORMAT: %s" % fmt,
                      "EDGE_WEIGHT_SECTION"] + body + ["EOF"]) + "\n"


@pytest.mark.parametrize("fmt", T.EXPLICIT_FORMATS)
def test_explicit_layouts(fmt):
    rng = np.random.default_rng(7)
    n = 9
    A = rng.integers(1, 100, size=(n, n))
    W = np.triu(A, 1)
    W = W + W.T
    got = T.parse_tsplib(_explicit_text(W, fmt))
    assert got.edge_weight_format == fmt
    assert np.array_equal(T.tsplib_weights(got), W)
    D = T.distance_matrix(got)
    assert D.dtype == np.float32 and np.array_equal(D, W.astype(np.float32))


def test_node_order_follows_the_indices_and_colon_spacing():
    xy = inst.uniform_cities(12, 5)
    order = [5, 0, 11, 3, 2, 1, 4, 6, 10, 9, 8, 7]
    a = T.parse_tsplib(_coord_text(xy, order=order, sep=": "))
    assert np.array_equal(a.coords, xy.astype(np.float64))


def test_round_trip_and_euclidean_metric_match_the_synthetic_generator():
    xy = inst.uniform_cities(50, 11)
    text = T.format_tsplib("u50", xy, comment="seeded uniform cities")
    got = T.parse_tsplib(text)
    assert got.name == "u50" and got.dimension == 50 and got.edge_weight_type == "EUC_2D"
    assert np.array_equal(got.coords, xy.astype(np.float64))
    # FP32 coordinates are exact in FP64: the same distances bit for bit
    assert np.array_equal(T.distance_matrix(got, "euclidean"), inst.distance_matrix(xy))


def test_tour_length_under_the_integer_metric():
    c = [(0.0, 0.0), (3.0, 0.0), (3.0, 4.0)]
    a = T.parse_tsplib(_coord_text(c))
    assert T.tour_length(a, [0, 1, 2]) == 12
    assert T.tour_length(a, [2, 0, 1]) == 12


def test_rejections():
    base = _coord_text([(0.0, 0.0), (3.0, 0.0), (3.0, 4.0)])
    with pytest.raises(T.TsplibError, match="ATSP"):
        T.parse_tsplib(base.replace("TYPE : TSP", "TYPE : ATSP"))
    with pytest.raises(T.TsplibError, match="GEO"):
        T.parse_tsplib(base.replace("EUC_2D", "GEO"))
    with pytest.raises(T.TsplibError, match="DIMENSION"):
        T.parse_tsplib(base.replace("DIMENSION : 3\n", ""))
    with pytest.raises(T.TsplibError, match="expected 12"):
        T.parse_tsplib(base.replace("DIMENSION : 3", "DIMENSION : 4"))
    with pytest.raises(T.TsplibError, match="at least 3"):
        T.parse_tsplib(_coord_text([(0.0, 0.0), (1.0, 0.0)]))
    with pytest.raises(T.TsplibError, match="not symmetric"):
        W = np.array([[0, 1, 2], [1, 0, 3], [2, 4, 0]])
        txt = _explicit_text(W, "FULL_MATRIX")
        T.parse_tsplib(txt)
    # duplicate points: a zero distance the method cannot take
    dup = T.parse_tsplib(_coord_text([(0.0, 0.0), (1.0, 0.0), (1.0, 0.0)]))
    with pytest.raises(T.TsplibError, match="nodes 2 and 3"):
        T.distance_matrix(dup)
    # close points that round to zero under EUC_2D but not in the plain metric
    close = T.parse_tsplib(_coord_text([(0.0, 0.0), (5.0, 0.0), (5.2, 0.0)]))
    with pytest.raises(T.TsplibError, match="tsplib metric"):
        T.distance_matrix(close)
    assert T.distance_matrix(close, "euclidean")[1, 2] > 0
    with pytest.raises(T.TsplibError, match="needs coordinates"):
        T.distance_matrix(T.parse_tsplib(_explicit_text(np.array([[0, 1, 2], [1, 0, 3], [2, 3, 0]]),
                                                        "UPPER_ROW")), "euclidean")


def test_instance_files(tmp_path):
    for name in ("b.tsp", "a.tsp", "notes.txt"):
        (tmp_path / name).write_text("x")
    files = T.instance_files([str(tmp_path)])
    assert [f.rsplit("/", 1)[1] for f in files] == ["a.tsp", "b.tsp"]
