"""CPU oracle for tensorized ACO on the Euclidean TSP.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product library never imports it.

Thin numpy wrappers over ``liboracle.so`` (built from ``aco_oracle.c`` by
``oracle/build.py``).  Every matrix is dense row-major n x n.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("ACO_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        sig = {
            "oracle_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
            "oracle_to_unit": (ctypes.c_float, [ctypes.c_uint32]),
            "oracle_uniform": (ctypes.c_float, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                                ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_start_city": (ctypes.c_int32, [ctypes.c_uint64, ctypes.c_uint32,
                                                   ctypes.c_uint32, ctypes.c_int32]),
            "oracle_transition": (None, [_f32p, _f32p, _f32p, ctypes.c_int32, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, _f32p]),
            "oracle_select": (ctypes.c_int32, [_f32p, _u8p, ctypes.c_int32, ctypes.c_uint64,
                                               ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_select_literal": (ctypes.c_int32, [_f64p, _u8p, ctypes.c_int32, ctypes.c_double,
                                                       ctypes.c_uint64, ctypes.c_uint32,
                                                       ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_tour_length": (ctypes.c_float, [_i32p, _f32p, ctypes.c_int32]),
            "oracle_construct": (None, [_f32p, _f32p, ctypes.c_int32, ctypes.c_uint64,
                                        ctypes.c_uint32, _i32p, ctypes.c_int32, _i32p, _f32p]),
            "oracle_length_lower_bound": (ctypes.c_double, [_f32p, ctypes.c_int32]),
            "oracle_deposit_scale": (ctypes.c_int32, [ctypes.c_double, ctypes.c_int32,
                                                      ctypes.c_float]),
            "oracle_deposit_weight": (ctypes.c_int64, [ctypes.c_float, ctypes.c_float,
                                                       ctypes.c_int32]),
            "oracle_elite": (None, [_f32p, ctypes.c_int32, ctypes.c_int32, _u8p]),
            "oracle_deposit": (None, [_i32p, _f32p, _u8p, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_float, ctypes.c_int32, _i64p]),
            "oracle_evaporate": (None, [_f32p, _i64p, ctypes.c_int32, ctypes.c_float,
                                        ctypes.c_int32]),
            "oracle_gamma": (ctypes.c_float, [ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                              ctypes.c_float]),
            "oracle_run": (ctypes.c_int32, [_f32p, _f32p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_uint64,
                                            ctypes.c_uint32, ctypes.c_int32, _f32p, _f32p,
                                            _i32p, _f32p, _i32p, _f32p]),
            "oracle_tsp_exact": (ctypes.c_double, [_f32p, ctypes.c_int32, _i32p]),
            "oracle_to_unit_many": (None, [_u32p, ctypes.c_int64, _f32p]),
            "oracle_mlp_param_count": (ctypes.c_int32, []),
            "oracle_bf16_round": (ctypes.c_float, [ctypes.c_float]),
            "oracle_edge_ranks": (None, [_f32p, ctypes.c_int32, _i32p]),
            "oracle_mean_nn": (ctypes.c_double, [_f32p, ctypes.c_int32]),
            "oracle_edge_features": (None, [_f32p, _i32p, ctypes.c_int32, ctypes.c_double,
                                            _f32p]),
            "oracle_mlp_forward": (None, [_f64p, _f32p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_double, ctypes.c_double, _f64p, _f64p]),
            "oracle_mlp_loss_grad": (ctypes.c_double, [_f64p, _f32p, _f32p, ctypes.c_int64,
                                                       ctypes.c_int32, _f64p]),
            "oracle_adam_step": (None, [_f64p, _f64p, _f64p, _f64p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double]),
            "oracle_transition_rows": (None, [_f32p, _f32p, _f32p, ctypes.c_int32, ctypes.c_float,
                                              ctypes.c_float, ctypes.c_float, _i32p,
                                              ctypes.c_int32, _f32p]),
            "oracle_clamp": (None, [_f32p, ctypes.c_int32, ctypes.c_float, ctypes.c_float]),
            "oracle_roulette_deviate": (ctypes.c_float, [ctypes.c_uint64, ctypes.c_uint32,
                                                         ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_select_roulette": (ctypes.c_int32, [_f32p, _u8p, ctypes.c_int32,
                                                        ctypes.c_uint64, ctypes.c_uint32,
                                                        ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_construct_roulette": (None, [_f32p, _f32p, ctypes.c_int32, ctypes.c_uint64,
                                                 ctypes.c_uint32, _i32p, ctypes.c_int32, _i32p,
                                                 _f32p]),
            "oracle_select_roulette_many": (None, [_f32p, _u8p, ctypes.c_int32, ctypes.c_uint64,
                                                   ctypes.c_uint32, ctypes.c_uint32,
                                                   ctypes.c_int32, _i32p]),
            "oracle_start_cities": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                           ctypes.c_int32, _i32p]),
            "oracle_select_many": (None, [_f32p, _f64p, _u8p, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_int32, _i32p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(arr, ctype):
    if arr is None:
        return None
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def _c(arr, dtype):
    return np.ascontiguousarray(arr, dtype=dtype)


def philox4x32_10(ctr, key):
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                               _ptr(out, ctypes.c_uint32))
    return out


def to_unit(w):
    return lib().oracle_to_unit(int(w) & 0xFFFFFFFF)


def uniform(seed, t, a, s, j):
    return lib().oracle_uniform(seed, t, a, s, j)


def start_city(seed, t, a, n):
    return lib().oracle_start_city(seed, t, a, n)


def transition(tau, dist, alpha, beta, gamma, eta=None):
    n = dist.shape[0]
    tau = _c(tau, np.float32)
    dist = _c(dist, np.float32)
    eta_c = None if eta is None else _c(eta, np.float32)
    P = np.zeros((n, n), np.float32)
    lib().oracle_transition(_ptr(tau, ctypes.c_float), _ptr(dist, ctypes.c_float),
                            _ptr(eta_c, ctypes.c_float), n, alpha, beta, gamma,
                            _ptr(P, ctypes.c_float))
    return P


def transition_rows(tau, dist, alpha, beta, gamma, rows, eta=None):
    """Rows `rows` of the transition matrix (len(rows) x n)."""
    n = dist.shape[0]
    tau = _c(tau, np.float32)
    dist = _c(dist, np.float32)
    eta_c = None if eta is None else _c(eta, np.float32)
    rows = _c(rows, np.int32)
    out = np.zeros((rows.shape[0], n), np.float32)
    lib().oracle_transition_rows(_ptr(tau, ctypes.c_float), _ptr(dist, ctypes.c_float),
                                 _ptr(eta_c, ctypes.c_float), n, alpha, beta, gamma,
                                 _ptr(rows, ctypes.c_int32), rows.shape[0],
                                 _ptr(out, ctypes.c_float))
    return out


def select(row, visited, seed, t, a, s):
    row = _c(row, np.float32)
    vis = None if visited is None else _c(visited, np.uint8)
    return lib().oracle_select(_ptr(row, ctypes.c_float), _ptr(vis, ctypes.c_uint8),
                               row.shape[0], seed, t, a, s)


def select_literal(p, visited, gamma, seed, t, a, s):
    p = _c(p, np.float64)
    vis = None if visited is None else _c(visited, np.uint8)
    return lib().oracle_select_literal(_ptr(p, ctypes.c_double), _ptr(vis, ctypes.c_uint8),
                                       p.shape[0], gamma, seed, t, a, s)


def tour_length(tour, dist):
    tour = _c(tour, np.int32)
    dist = _c(dist, np.float32)
    return lib().oracle_tour_length(_ptr(tour, ctypes.c_int32), _ptr(dist, ctypes.c_float),
                                    dist.shape[0])


def construct(P, dist, seed, t, ants, *, selection="adair"):
    """Tours and lengths of the given ants; selection "adair" (argmax of
    P * r, Sec. 2.4) or "roulette" (the Roulette Wheel baseline)."""
    n = dist.shape[0]
    P = _c(P, np.float32)
    dist = _c(dist, np.float32)
    ants = _c(ants, np.int32)
    tours = np.zeros((ants.shape[0], n), np.int32)
    lengths = np.zeros(ants.shape[0], np.float32)
    fn = {"adair": lib().oracle_construct, "roulette": lib().oracle_construct_roulette}[selection]
    fn(_ptr(P, ctypes.c_float), _ptr(dist, ctypes.c_float), n, seed, t,
       _ptr(ants, ctypes.c_int32), ants.shape[0], _ptr(tours, ctypes.c_int32),
       _ptr(lengths, ctypes.c_float))
    return tours, lengths


def clamp(tau, tau_min, tau_max):
    """MAX-MIN bounds applied to a copy of tau (off the diagonal)."""
    tau = np.array(tau, dtype=np.float32, copy=True, order="C")
    lib().oracle_clamp(_ptr(tau, ctypes.c_float), tau.shape[0], tau_min, tau_max)
    return tau


def roulette_deviate(seed, t, a, s):
    return lib().oracle_roulette_deviate(seed, t, a, s)


def select_roulette(row, visited, seed, t, a, s):
    row = _c(row, np.float32)
    vis = None if visited is None else _c(visited, np.uint8)
    return lib().oracle_select_roulette(_ptr(row, ctypes.c_float), _ptr(vis, ctypes.c_uint8),
                                        row.shape[0], seed, t, a, s)


def select_roulette_many(row, visited, seed, t, s, count):
    """count ants (a = 0..count-1) each take one Roulette Wheel step from the same row."""
    row = _c(row, np.float32)
    vis = None if visited is None else _c(visited, np.uint8)
    out = np.zeros(count, np.int32)
    lib().oracle_select_roulette_many(_ptr(row, ctypes.c_float), _ptr(vis, ctypes.c_uint8),
                                      row.shape[0], seed, t, s, count, _ptr(out, ctypes.c_int32))
    return out


def length_lower_bound(dist):
    dist = _c(dist, np.float32)
    return lib().oracle_length_lower_bound(_ptr(dist, ctypes.c_float), dist.shape[0])


def deposit_scale(dist, m_max, Q):
    return lib().oracle_deposit_scale(length_lower_bound(dist), m_max, Q)


def deposit_weight(length, Q, S):
    return lib().oracle_deposit_weight(length, Q, S)


def elite(lengths, k):
    lengths = _c(lengths, np.float32)
    out = np.zeros(lengths.shape[0], np.uint8)
    lib().oracle_elite(_ptr(lengths, ctypes.c_float), lengths.shape[0], k,
                       _ptr(out, ctypes.c_uint8))
    return out


def deposit(tours, lengths, elite_mask, Q, S):
    tours = _c(tours, np.int32)
    lengths = _c(lengths, np.float32)
    m, n = tours.shape
    em = None if elite_mask is None else _c(elite_mask, np.uint8)
    delta = np.zeros((n, n), np.int64)
    lib().oracle_deposit(_ptr(tours, ctypes.c_int32), _ptr(lengths, ctypes.c_float),
                         _ptr(em, ctypes.c_uint8), m, n, Q, S, _ptr(delta, ctypes.c_int64))
    return delta


def evaporate(tau, delta, rho, S):
    tau = np.array(tau, dtype=np.float32, copy=True, order="C")
    d = None if delta is None else _c(delta, np.int64)
    lib().oracle_evaporate(_ptr(tau, ctypes.c_float), _ptr(d, ctypes.c_int64),
                           tau.shape[0], rho, S)
    return tau


def gamma(t, T, gamma_max, gamma_min):
    return lib().oracle_gamma(t, T, gamma_max, gamma_min)


def run(dist, m, alpha, beta, rho, Q, seed, iters, *, m_max=None, elite_k=0,
        gamma_max=1.5, gamma_min=1.0, tau0=1.0, iter0=0, eta=None, tau=None,
        selection="adair", tau_min=0.0, tau_max=float("inf")):
    """Whole run; returns dict(tau, P, best_tour, best_len, best_iter, S, iter_best)."""
    n = dist.shape[0]
    dist = _c(dist, np.float32)
    eta_c = None if eta is None else _c(eta, np.float32)
    if tau is None:
        tau = np.full((n, n), tau0, np.float32)
        np.fill_diagonal(tau, 0.0)
    tau = np.array(tau, dtype=np.float32, copy=True, order="C")
    P = np.zeros((n, n), np.float32)
    best_tour = np.zeros(n, np.int32)
    best_len = ctypes.c_float()
    best_iter = ctypes.c_int32()
    iter_best = np.zeros(max(iters, 1), np.float32)
    S = lib().oracle_run(_ptr(dist, ctypes.c_float), _ptr(eta_c, ctypes.c_float), n, m,
                         m if m_max is None else m_max, alpha, beta, rho, Q, elite_k,
                         gamma_max, gamma_min, {"adair": 0, "roulette": 1}[selection],
                         tau_min, tau_max, seed, iter0, iters, _ptr(tau, ctypes.c_float),
                         _ptr(P, ctypes.c_float), _ptr(best_tour, ctypes.c_int32),
                         ctypes.byref(best_len), ctypes.byref(best_iter),
                         _ptr(iter_best, ctypes.c_float))
    if S < 0:
        raise MemoryError("oracle_run: allocation failed")
    return dict(tau=tau, P=P, best_tour=best_tour, best_len=best_len.value,
                best_iter=best_iter.value, S=S, iter_best=iter_best[:iters])


def tsp_exact(dist):
    dist = _c(dist, np.float32)
    tour = np.zeros(dist.shape[0], np.int32)
    L = lib().oracle_tsp_exact(_ptr(dist, ctypes.c_float), dist.shape[0],
                               _ptr(tour, ctypes.c_int32))
    return L, tour


def to_unit_many(words):
    w = _c(words, np.uint32)
    out = np.zeros(w.shape[0], np.float32)
    lib().oracle_to_unit_many(_ptr(w, ctypes.c_uint32), w.shape[0], _ptr(out, ctypes.c_float))
    return out


def start_cities(seed, t, n, count):
    out = np.zeros(count, np.int32)
    lib().oracle_start_cities(seed, t, n, count, _ptr(out, ctypes.c_int32))
    return out


def select_many(row, visited, seed, t, s, count, *, gamma=1.0, literal=False):
    """count ants (a = 0..count-1) each take one step from the same row.

    literal=False: row is P with the 1/gamma exponent folded in.
    literal=True:  row is the row-normalised M_p; score p * u**gamma in FP64.
    """
    n = len(row)
    vis = None if visited is None else _c(visited, np.uint8)
    out = np.zeros(count, np.int32)
    if literal:
        p = _c(row, np.float64)
        lib().oracle_select_many(None, _ptr(p, ctypes.c_double), _ptr(vis, ctypes.c_uint8), n,
                                 gamma, 1, seed, t, s, count, _ptr(out, ctypes.c_int32))
    else:
        r = _c(row, np.float32)
        lib().oracle_select_many(_ptr(r, ctypes.c_float), None, _ptr(vis, ctypes.c_uint8), n,
                                 gamma, 0, seed, t, s, count, _ptr(out, ctypes.c_int32))
    return out


# ---------------------------------------------------------------------------
# learned edge heuristic (mlp_oracle.c)
# ---------------------------------------------------------------------------
def mlp_param_count():
    return lib().oracle_mlp_param_count()


def bf16_round(x):
    return lib().oracle_bf16_round(float(x))


def edge_ranks(dist):
    dist = _c(dist, np.float32)
    n = dist.shape[0]
    rank = np.zeros((n, n), np.int32)
    lib().oracle_edge_ranks(_ptr(dist, ctypes.c_float), n, _ptr(rank, ctypes.c_int32))
    return rank


def mean_nn(dist):
    dist = _c(dist, np.float32)
    return lib().oracle_mean_nn(_ptr(dist, ctypes.c_float), dist.shape[0])


def edge_features(dist, rank=None, mean=None):
    """(n, n, 3) float32 features; the diagonal is zero."""
    dist = _c(dist, np.float32)
    n = dist.shape[0]
    rank = edge_ranks(dist) if rank is None else _c(rank, np.int32)
    mean = mean_nn(dist) if mean is None else float(mean)
    feats = np.zeros((n, n, 3), np.float32)
    lib().oracle_edge_features(_ptr(dist, ctypes.c_float), _ptr(rank, ctypes.c_int32), n, mean,
                               _ptr(feats, ctypes.c_float))
    return feats


def mlp_forward(params, feats, round_bf16=True, kappa=1.0, lam=0.0):
    """(z, eta) for (count, 3) features; eta = sigmoid(z)^kappa / f1^lam."""
    params = _c(params, np.float64)
    feats = _c(feats, np.float32).reshape(-1, 3)
    z = np.zeros(feats.shape[0], np.float64)
    eta = np.zeros(feats.shape[0], np.float64)
    lib().oracle_mlp_forward(_ptr(params, ctypes.c_double), _ptr(feats, ctypes.c_float),
                             feats.shape[0], 1 if round_bf16 else 0, kappa, lam,
                             _ptr(z, ctypes.c_double), _ptr(eta, ctypes.c_double))
    return z, eta


def mlp_loss_grad(params, feats, y, round_bf16=True):
    params = _c(params, np.float64)
    feats = _c(feats, np.float32).reshape(-1, 3)
    y = _c(y, np.float32)
    grad = np.zeros(mlp_param_count(), np.float64)
    loss = lib().oracle_mlp_loss_grad(_ptr(params, ctypes.c_double), _ptr(feats, ctypes.c_float),
                                      _ptr(y, ctypes.c_float), feats.shape[0],
                                      1 if round_bf16 else 0, _ptr(grad, ctypes.c_double))
    return loss, grad


def adam_step(params, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float64 arrays params, m, v."""
    g = _c(grad, np.float64)
    lib().oracle_adam_step(_ptr(params, ctypes.c_double), _ptr(m, ctypes.c_double),
                           _ptr(v, ctypes.c_double), _ptr(g, ctypes.c_double), params.shape[0],
                           t, lr, b1, b2, eps)
