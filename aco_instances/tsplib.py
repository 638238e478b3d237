"""Reader (and writer) for symmetric TSP instances in the TSPLIB format.

Inputs only, like the rest of this package: it turns a TSPLIB file into the
FP32 distance matrix the library and the oracle take, and holds none of the
ACO arithmetic.  The paper's runtime and convergence experiments (Sec. 3) use
TSPLIB instances; with the files at hand, `scaling.py --tsplib` and
`ablation.py --tsplib` run on them instead of the synthetic stand-ins.

Supported (the keywords of the TSPLIB format description, Reinelt 1991):
  TYPE: TSP
  EDGE_WEIGHT_TYPE: EUC_2D, CEIL_2D, ATT (NODE_COORD_SECTION, 2-D), or
                    EXPLICIT with EDGE_WEIGHT_FORMAT FULL_MATRIX, UPPER_ROW,
                    LOWER_ROW, UPPER_DIAG_ROW, LOWER_DIAG_ROW, UPPER_COL,
                    LOWER_COL, UPPER_DIAG_COL or LOWER_DIAG_COL.
Other types (GEO, EUC_3D, MAN_2D, ...) and other problems (ATSP, HCP, ...)
are rejected with an error naming them.

Two metrics:
  "tsplib"    -- the file's own integer distance function, as TSPLIB defines
                 it (the lengths its published optimal tours refer to):
                 EUC_2D rounds the Euclidean distance to the nearest integer,
                 CEIL_2D rounds it up, ATT is the pseudo-Euclidean distance
                 (sqrt of the squared distance over 10, rounded up when
                 rounding to nearest fell below it); EXPLICIT takes the
                 given weights.
  "euclidean" -- the plain Euclidean distance of the coordinates in FP64,
                 rounded once to FP32 (coordinate files only).
The ACO needs positive off-diagonal distances (eta = 1/d); a matrix with a
zero or negative one (duplicate points, or close points under rounding) is
rejected, naming the pair.
"""
from __future__ import annotations

import dataclasses
import os

import numpy as np

COORD_TYPES = ("EUC_2D", "CEIL_2D", "ATT")
EXPLICIT_FORMATS = ("FULL_MATRIX", "UPPER_ROW", "LOWER_ROW", "UPPER_DIAG_ROW", "LOWER_DIAG_ROW",
                    "UPPER_COL", "LOWER_COL", "UPPER_DIAG_COL", "LOWER_DIAG_COL")


class TsplibError(ValueError):
    pass


@dataclasses.dataclass
class TsplibInstance:
    name: str
    dimension: int
    edge_weight_type: str
    coords: np.ndarray | None        # n x 2 float64 (coordinate types)
    weights: np.ndarray | None       # n x n int64 or float64 (EXPLICIT)
    edge_weight_format: str | None = None
    comment: str = ""


def _split_spec(line):
    key, _, value = line.partition(":")
    return key.strip().upper(), value.strip()


def parse_tsplib(text: str) -> TsplibInstance:
    """Parse the text of a TSPLIB file."""
    spec = {}
    numbers = {}  # section name -> list of tokens
    section = None
    for raw in text.splitlines():
        line = raw.strip()
        if not line:
            continue
        upper = line.upper()
        if upper == "EOF":
            break
        if upper.endswith("_SECTION"):
            section = upper
            numbers.setdefault(section, [])
            continue
        if section is not None and ":" not in line:
            numbers[section].extend(line.split())
            continue
        key, value = _split_spec(line)
        if key.endswith("_SECTION"):  # "NODE_COORD_SECTION :" with a colon
            section = key
            numbers.setdefault(section, [])
            if value:
                numbers[section].extend(value.split())
            continue
        section = None
        spec[key] = value
    kind = spec.get("TYPE", "").upper()
    if kind != "TSP":
        raise TsplibError("TYPE %r is not supported (symmetric TSP only)" % (kind or "missing"))
    if "DIMENSION" not in spec:
        raise TsplibError("no DIMENSION")
    n = int(spec["DIMENSION"])
    if n < 3:
        raise TsplibError("DIMENSION %d: the method needs at least 3 cities" % n)
    ewt = spec.get("EDGE_WEIGHT_TYPE", "").upper()
    name = spec.get("NAME", "")
    comment = spec.get("COMMENT", "")
    if ewt in COORD_TYPES:
        toks = numbers.get("NODE_COORD_SECTION")
        if toks is None:
            raise TsplibError("%s needs a NODE_COORD_SECTION" % ewt)
        if len(toks) != 3 * n:
            raise TsplibError("NODE_COORD_SECTION holds %d numbers, expected %d (index, x, y "
                              "for %d nodes)" % (len(toks), 3 * n, n))
        rows = np.array(toks, dtype=np.float64).reshape(n, 3)
        index = rows[:, 0].astype(np.int64)
        if not np.array_equal(np.sort(index), np.arange(1, n + 1)):
            raise TsplibError("node indices are not 1..%d" % n)
        coords = np.empty((n, 2), np.float64)
        coords[index - 1] = rows[:, 1:]
        return TsplibInstance(name, n, ewt, coords, None, None, comment)
    if ewt == "EXPLICIT":
        fmt = spec.get("EDGE_WEIGHT_FORMAT", "").upper()
        if fmt not in EXPLICIT_FORMATS:
            raise TsplibError("EDGE_WEIGHT_FORMAT %r is not supported" % (fmt or "missing"))
        toks = numbers.get("EDGE_WEIGHT_SECTION")
        if toks is None:
            raise TsplibError("EXPLICIT needs an EDGE_WEIGHT_SECTION")
        vals = np.array(toks, dtype=np.float64)
        return TsplibInstance(name, n, ewt, None, _explicit_matrix(vals, n, fmt), fmt, comment)
    raise TsplibError("EDGE_WEIGHT_TYPE %r is not supported" % (ewt or "missing"))


def _explicit_matrix(vals, n, fmt):
    """The full symmetric matrix from an EDGE_WEIGHT_SECTION.  A *_COL format
    lists the transpose's entries in the order of the matching *_ROW format,
    which for a symmetric matrix is the other triangle."""
    if fmt == "FULL_MATRIX":
        if vals.size != n * n:
            raise TsplibError("FULL_MATRIX holds %d numbers, expected %d" % (vals.size, n * n))
        W = vals.reshape(n, n)
        if not np.array_equal(W, W.T):
            raise TsplibError("FULL_MATRIX is not symmetric")
        return W
    row_of_col = {"UPPER_COL": "LOWER_ROW", "LOWER_COL": "UPPER_ROW",
                  "UPPER_DIAG_COL": "LOWER_DIAG_ROW", "LOWER_DIAG_COL": "UPPER_DIAG_ROW"}
    fmt = row_of_col.get(fmt, fmt)
    k = 0 if "DIAG" in fmt else 1
    # the triangle's (row, column) pairs in row-major order
    rows, cols = np.triu_indices(n, k) if fmt.startswith("UPPER") else np.tril_indices(n, -k)
    if vals.size != rows.size:
        raise TsplibError("%s holds %d numbers, expected %d" % (fmt, vals.size, rows.size))
    W = np.zeros((n, n), np.float64)
    W[rows, cols] = vals
    W[cols, rows] = vals
    return W


def read_tsplib(path: str) -> TsplibInstance:
    with open(path) as f:
        return parse_tsplib(f.read())


def _nint(x):
    """Nearest integer, halves up: the rounding TSPLIB's distance functions use."""
    return np.floor(x + 0.5)


def tsplib_weights(inst: TsplibInstance) -> np.ndarray:
    """The instance's integer distance function as an n x n int64 matrix
    (zero diagonal)."""
    if inst.weights is not None:
        W = inst.weights.copy()
    else:
        x, y = inst.coords[:, 0], inst.coords[:, 1]
        dx = x[:, None] - x[None, :]
        dy = y[:, None] - y[None, :]
        sq = dx * dx + dy * dy
        if inst.edge_weight_type == "EUC_2D":
            W = _nint(np.sqrt(sq))
        elif inst.edge_weight_type == "CEIL_2D":
            W = np.ceil(np.sqrt(sq))
        else:  # ATT
            r = np.sqrt(sq / 10.0)
            t = _nint(r)
            W = np.where(t < r, t + 1.0, t)
    np.fill_diagonal(W, 0.0)
    return W.astype(np.int64)


def distance_matrix(inst: TsplibInstance, metric: str = "tsplib") -> np.ndarray:
    """FP32 n x n distances for the library and the oracle (zero diagonal).
    Raises TsplibError if an off-diagonal distance is not positive."""
    if metric == "tsplib":
        D = tsplib_weights(inst).astype(np.float64)
    elif metric == "euclidean":
        if inst.coords is None:
            raise TsplibError("the euclidean metric needs coordinates; %s has none"
                              % (inst.name or "this instance"))
        x, y = inst.coords[:, 0], inst.coords[:, 1]
        dx = x[:, None] - x[None, :]
        dy = y[:, None] - y[None, :]
        D = np.sqrt(dx * dx + dy * dy)
    else:
        raise TsplibError("metric %r: use 'tsplib' or 'euclidean'" % metric)
    D = D.astype(np.float32)
    np.fill_diagonal(D, 0.0)
    off = ~np.eye(D.shape[0], dtype=bool)
    bad = np.argwhere(off & ~(D > 0))
    if bad.size:
        i, j = (int(v) for v in bad[0])
        raise TsplibError("distance between nodes %d and %d is %g under the %s metric; the "
                          "method needs positive distances" % (i + 1, j + 1, D[i, j], metric))
    return D


def tour_length(inst: TsplibInstance, tour) -> int:
    """Closed length of a tour (0-based city order) under the instance's own
    integer metric, for comparison with published optimal lengths."""
    W = tsplib_weights(inst)
    t = np.asarray(tour, dtype=np.int64)
    return int(W[t, np.roll(t, -1)].sum())


def format_tsplib(name: str, coords: np.ndarray, edge_weight_type: str = "EUC_2D",
                  comment: str = "") -> str:
    """TSPLIB text of a coordinate instance (for synthetic instances)."""
    if edge_weight_type not in COORD_TYPES:
        raise TsplibError("EDGE_WEIGHT_TYPE %r is not a coordinate type" % edge_weight_type)
    lines = ["NAME : %s" % name, "TYPE : TSP"]
    if comment:
        lines.append("COMMENT : %s" % comment)
    lines += ["DIMENSION : %d" % coords.shape[0], "EDGE_WEIGHT_TYPE : %s" % edge_weight_type,
              "NODE_COORD_SECTION"]
    lines += ["%d %s %s" % (i + 1, repr(float(x)), repr(float(y)))
              for i, (x, y) in enumerate(coords)]
    lines.append("EOF")
    return "\n".join(lines) + "\n"


def instance_files(paths):
    """Expand files and directories (every *.tsp inside) into a sorted list."""
    out = []
    for p in paths:
        if os.path.isdir(p):
            out += sorted(os.path.join(p, f) for f in os.listdir(p) if f.lower().endswith(".tsp"))
        else:
            out.append(p)
    return out


__all__ = ["TsplibError", "TsplibInstance", "parse_tsplib", "read_tsplib", "tsplib_weights",
           "distance_matrix", "tour_length", "format_tsplib", "instance_files"]
