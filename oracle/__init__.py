"""Plain CPU oracle for random hyperbolic graph generation (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never loads it, and it never loads
the product library: the two share no code.  See ``rhg_oracle.c`` for what is
computed and which passage of the paper each step follows.

The binding is argument marshalling only (numpy arrays in, numpy arrays out);
every step of the computation runs in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rhg_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "librhg_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64 + binary128, OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = C.CDLL(_LIB_PATH)
        d, i64, u64, i32 = C.c_double, C.c_int64, C.c_uint64, C.c_int
        pd, pi64, pi32, pu32 = (C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int32), C.POINTER(C.c_uint32))
        lib.orc_philox4x32_10.argtypes = [pu32, pu32, pu32]
        lib.orc_uniforms.argtypes = [u64, i64, pd, pd]
        lib.orc_alpha.restype = d
        lib.orc_alpha.argtypes = [d]
        lib.orc_kbar_eq22.restype = d
        lib.orc_kbar_eq22.argtypes = [d, d, d, i32]
        lib.orc_kbar_minus.restype = d
        lib.orc_kbar_minus.argtypes = [d, d, d, d]
        lib.orc_solve_R.restype = i32
        lib.orc_solve_R.argtypes = [d, d, d, pd, pd]
        lib.orc_cosh.restype = d
        lib.orc_cosh.argtypes = [d]
        lib.orc_radius.restype = d
        lib.orc_radius.argtypes = [d, d, d, C.POINTER(C.c_int)]
        lib.orc_sample.restype = i64
        lib.orc_sample.argtypes = [u64, d, d, i64, i64, pd, pd, i32]
        lib.orc_is_edge.restype = i32
        lib.orc_is_edge.argtypes = [d, d, d, d, d, pi64]
        lib.orc_is_edge_quad.restype = i32
        lib.orc_is_edge_quad.argtypes = [d, d, d, d, d]
        lib.orc_is_edge_literal.restype = i32
        lib.orc_is_edge_literal.argtypes = [d, d, d, d, d]
        lib.orc_lr_candidates.argtypes = [u64, i64, i64, i64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        lib.orc_degrees.argtypes = [i64, pd, pd, d, pi32, i32, pi64]
        lib.orc_csr_fill.argtypes = [i64, pd, pd, d, pi64, pi32, i32]
        lib.orc_rows.restype = i64
        lib.orc_rows.argtypes = [i64, pd, pd, d, pi64, i64, pi64, pi32, i64, i32, pi64]
        lib.orc_max_threads.restype = i32
        lib.orc_mix64.restype = u64
        lib.orc_mix64.argtypes = [u64]
        lib.orc_pair_scan.argtypes = [i64, pd, pd, d, pi32, C.POINTER(C.c_uint64), i32, pi64, pd]
        lib.orc_temp_coin.restype = u64
        lib.orc_temp_coin.argtypes = [u64, i64, i64]
        lib.orc_temp_is_edge.argtypes = [d, d, d, d, d, d, u64, pi64]
        lib.orc_temp_is_edge_quad.argtypes = [d, d, d, d, d, d, u64]
        lib.orc_temp_edges.restype = i64
        lib.orc_temp_edges.argtypes = [i64, pd, pd, d, d, u64, pi64, pi64, i64, i32, pi64]
        lib.orc_temp_rows.restype = i64
        lib.orc_temp_rows.argtypes = [i64, pd, pd, d, d, u64, pi64, i64, pi64, pi32, i64, i32, pi64]
        _lib = lib
        return lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def threads() -> int:
    return int(_load().orc_max_threads())


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def uniforms(seed: int, i: int):
    lib = _load()
    a, b = C.c_double(), C.c_double()
    lib.orc_uniforms(seed, i, C.byref(a), C.byref(b))
    return a.value, b.value


def alpha(gamma: float) -> float:
    return float(_load().orc_alpha(gamma))


def kbar_eq22(n: float, alpha_: float, R: float, literal: bool = False) -> float:
    return float(_load().orc_kbar_eq22(float(n), alpha_, R, 1 if literal else 0))


def kbar_minus(n: float, alpha_: float, R: float, target: float) -> float:
    """Eq. (22) minus target, differenced in binary128."""
    return float(_load().orc_kbar_minus(float(n), alpha_, R, target))


def solve_R(n: int, kbar: float, gamma: float):
    """Return (alpha, R) or raise ValueError when no root exists."""
    lib = _load()
    a, r = C.c_double(), C.c_double()
    if lib.orc_solve_R(float(n), kbar, gamma, C.byref(a), C.byref(r)) != 0:
        raise ValueError("no radius on the decreasing branch of Eq. (22)")
    return a.value, r.value


def cosh(x: float) -> float:
    return float(_load().orc_cosh(x))


def radius(u: float, alpha_: float, R: float):
    """Correctly rounded inverse-CDF radius for one uniform: (r, near_midpoint)."""
    h = C.c_int()
    r = _load().orc_radius(u, alpha_, R, C.byref(h))
    return float(r), bool(h.value)


def sample(seed: int, alpha_: float, R: float, n: int, i0: int = 0, nthreads: int = 0):
    """Points i0 .. i0+n-1: returns (r, theta, near_midpoint_count)."""
    lib = _load()
    r = np.empty(n, dtype=np.float64)
    t = np.empty(n, dtype=np.float64)
    hard = lib.orc_sample(seed, alpha_, R, i0, n, _p(r, C.c_double), _p(t, C.c_double), nthreads)
    return r, t, int(hard)


def is_edge(ri, ti, rj, tj, R):
    st = np.zeros(2, dtype=np.int64)
    e = _load().orc_is_edge(ri, ti, rj, tj, R, _p(st, C.c_int64))
    return bool(e), int(st[0]), int(st[1])


def is_edge_literal(ri, ti, rj, tj, R):
    """The printed cosh-distance law evaluated literally in binary64
    (diagnostic: it loses the decision near the rim at large R)."""
    return bool(_load().orc_is_edge_literal(ri, ti, rj, tj, R))


def is_edge_quad(ri, ti, rj, tj, R):
    return bool(_load().orc_is_edge_quad(ri, ti, rj, tj, R))


def degrees(r, theta, R, nthreads: int = 0):
    """Degrees by brute force over all pairs; returns (deg, quad_fallbacks, ties)."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = r.shape[0]
    deg = np.zeros(n, dtype=np.int32)
    st = np.zeros(2, dtype=np.int64)
    lib.orc_degrees(n, _p(r, C.c_double), _p(theta, C.c_double), R, _p(deg, C.c_int32),
                    nthreads, _p(st, C.c_int64))
    return deg, int(st[0]), int(st[1])


def csr(r, theta, R, nthreads: int = 0):
    """Symmetric CSR (int64 row_ptr, int32 col) with ascending rows, plus stats."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    deg, nq, nt = degrees(r, theta, R, nthreads)
    n = r.shape[0]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    lib.orc_csr_fill(n, _p(r, C.c_double), _p(theta, C.c_double), R, _p(row_ptr, C.c_int64),
                     _p(col, C.c_int32), nthreads)
    return row_ptr, col, nq, nt


def rows(r, theta, R, which, nthreads: int = 0):
    """Ascending neighbour lists of the vertices in ``which``, each tested
    against all n points: returns (ptr, col, quad_fallbacks, ties)."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    which = np.ascontiguousarray(which, dtype=np.int64)
    n = r.shape[0]
    cap = 1 << 16
    while True:
        ptr = np.zeros(which.shape[0] + 1, dtype=np.int64)
        col = np.empty(cap, dtype=np.int32)
        st = np.zeros(2, dtype=np.int64)
        tot = lib.orc_rows(n, _p(r, C.c_double), _p(theta, C.c_double), R, _p(which, C.c_int64),
                           which.shape[0], _p(ptr, C.c_int64), _p(col, C.c_int32), cap, nthreads,
                           _p(st, C.c_int64))
        if tot >= 0:
            return ptr, col[:tot].copy(), int(st[0]), int(st[1])
        cap = int(ptr[-1]) + 1


def mix64(z: int) -> int:
    """SplitMix64's finaliser (the fingerprint's hash of one packed pair)."""
    return int(_load().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def pair_scan(r, theta, R, nthreads: int = 0, timing: bool = False):
    """Every pair i < j tested once, nothing stored: returns (deg, fp_sum,
    fp_xor, quad_fallbacks, ties), the fingerprint being the wrapping sum and
    the xor of mix64(i * 2^32 + j) over the edges; with timing=True also the
    wall time of the pair loop alone, in seconds."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = r.shape[0]
    deg = np.zeros(n, dtype=np.int32)
    fp = np.zeros(2, dtype=np.uint64)
    st = np.zeros(2, dtype=np.int64)
    loop = np.zeros(1, dtype=np.float64)
    lib.orc_pair_scan(n, _p(r, C.c_double), _p(theta, C.c_double), R, _p(deg, C.c_int32),
                      _p(fp, C.c_uint64), nthreads, _p(st, C.c_int64), _p(loop, C.c_double))
    out = (deg, int(fp[0]), int(fp[1]), int(st[0]), int(st[1]))
    return out + (float(loop[0]),) if timing else out


def generate(n: int, kbar: float, gamma: float, seed: int, nthreads: int = 0):
    """Whole oracle pipeline: (alpha, R, r, theta, row_ptr, col, stats dict)."""
    a, R = solve_R(n, kbar, gamma)
    r, t, hard = sample(seed, a, R, n, nthreads=nthreads)
    row_ptr, col, nq, nt = csr(r, t, R, nthreads)
    return a, R, r, t, row_ptr, col, {"near_midpoint": hard, "quad": nq, "ties": nt}


# --------------------------------------------------------------------------
# Long-range augmentation (RHG-LR): the paper adds a small share (0.5 % in
# its experiment) of edges between vertex pairs drawn uniformly at random
# to correct the diameter (Sec. 4.2, comparison with real-world networks;
# RHG-LR in the generator table of Sec. 4.3; Appendix I).  Definition used
# here, in plain sequential form:
#   candidate j = 0, 1, 2, ... is the pair orc_lr_candidates(seed, j);
#   it is rejected if it is a self-loop, an edge of the graph, or a pair an
#   earlier candidate already added; the first k accepted are added, and at
#   most the candidates j < 2k + 4096 are drawn (fewer than k are added only
#   when more than half of the drawn pairs are rejected, i.e. in very dense
#   or tiny graphs).
# --------------------------------------------------------------------------

def lr_candidates(seed: int, j0: int, count: int, n: int):
    lib = _load()
    a = np.empty(max(count, 0), dtype=np.int64)
    b = np.empty(max(count, 0), dtype=np.int64)
    if count > 0:
        lib.orc_lr_candidates(seed, j0, count, n, _p(a, C.c_int64), _p(b, C.c_int64))
    return a, b


def lr_draw_limit(k: int) -> int:
    return 2 * k + 4096


def lr_added_pairs(n: int, row_ptr, col, k: int, seed: int):
    """The accepted candidates, in order, as a list of (a, b), a < b."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    ca, cb = lr_candidates(seed, 0, lr_draw_limit(k), n)
    # membership of every candidate in the graph (ordered pairs a < b)
    in_graph = np.isin(ca * n + cb, src * n + col)
    seen, added = set(), []
    for a, b, e in zip(ca.tolist(), cb.tolist(), in_graph.tolist()):
        if len(added) == k:
            break
        key = a * n + b
        if a == b or e or key in seen:
            continue
        seen.add(key)
        added.append((a, b))
    return added


def lr_augment(n: int, row_ptr, col, k: int, seed: int):
    """The augmented CSR: each row is the given row followed by its added
    neighbours in the order their pairs were accepted."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int32)
    added = lr_added_pairs(n, row_ptr, col, k, seed)
    extra = {}
    for a, b in added:
        extra.setdefault(a, []).append(b)
        extra.setdefault(b, []).append(a)
    cnt = np.zeros(n, dtype=np.int64)
    for v, lst in extra.items():
        cnt[v] = len(lst)
    out_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.diff(row_ptr) + cnt, out=out_ptr[1:])
    out = np.empty(int(out_ptr[-1]), dtype=np.int32)
    # every row: its old entries, then its added neighbours
    shift = out_ptr[:-1] - row_ptr[:-1]
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    out[np.arange(col.size, dtype=np.int64) + shift[src]] = col
    for v, lst in extra.items():
        end = out_ptr[v] + (row_ptr[v + 1] - row_ptr[v])
        out[end:end + len(lst)] = lst
    return out_ptr, out, len(added)


# --------------------------------------------------------------------------
# Graph statistics used to validate generated graphs (Sec. 4.1): the degree
# distribution and its power-law exponent, degree assortativity, and the
# clustering coefficient as the fraction of closed triangles to triads
# (paths of length 2).  Plain numpy / scipy on the host.
# --------------------------------------------------------------------------

def graph_stats(row_ptr, col, kmin: float = 10.0, triangles: bool = True) -> dict:
    """row_ptr, col: a simple symmetric CSR.  Returns
      hist[b]: vertices of degree 0 (b = 0) and of degree in [2^(b-1), 2^b)
               (b = 1 .. 32);
      gamma_mle: the discrete power-law maximum-likelihood exponent of the
               degrees k >= kmin in its usual approximation,
               1 + N / sum ln(k / (kmin - 1/2)) (Clauset, Shalizi, Newman,
               "Power-law distributions in empirical data", 2009);
      assortativity: Pearson correlation of the degrees at the two ends of
               the edges (Newman 2002), over both directions of every edge;
      triangles, triads = sum C(d, 2), transitivity = 3 triangles / triads,
      avg_local_clustering: mean over vertices of degree >= 2 of
               t(v) / C(d(v), 2), t(v) the triangles through v."""
    import scipy.sparse as sp
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    deg = np.diff(row_ptr)
    out = {"n": n, "nnz": int(row_ptr[-1]), "max_degree": int(deg.max()) if n else 0}
    hist = np.zeros(33, dtype=np.int64)
    hist[0] = int(np.sum(deg == 0))
    pos = deg[deg > 0]
    b = np.floor(np.log2(pos.astype(np.float64))).astype(np.int64) + 1 if pos.size else pos
    np.add.at(hist, b, 1)
    out["hist"] = hist
    tail = deg[deg >= kmin].astype(np.float64)
    out["tail_count"] = int(tail.size)
    out["gamma_mle"] = float(1.0 + tail.size / np.sum(np.log(tail / (kmin - 0.5)))) if tail.size else float("nan")
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    x = deg[src].astype(np.float64)
    y = deg[col].astype(np.float64)
    if x.size:
        mx = x.mean()
        var = (x * x).mean() - mx * mx
        out["assortativity"] = float(((x * y).mean() - mx * y.mean()) / var) if var > 0 else float("nan")
    else:
        out["assortativity"] = float("nan")
    d = deg.astype(np.int64)
    triads = int(np.sum(d * (d - 1) // 2))
    out["triads"] = triads
    if triangles:
        A = sp.csr_matrix((np.ones(col.size, dtype=np.int64), col, row_ptr), shape=(n, n))
        # t(v) = (1/2) sum_{u,w} A_vu A_uw A_wv
        t = np.asarray((A @ A).multiply(A).sum(axis=1)).ravel() // 2
        T = int(t.sum()) // 3
        out["triangles"] = T
        out["transitivity"] = 3.0 * T / triads if triads else float("nan")
        ok = d >= 2
        out["avg_local_clustering"] = float(np.mean(t[ok] / (d[ok] * (d[ok] - 1) / 2.0))) if ok.any() else float("nan")
        out["vertex_triangles"] = t
    return out


# --------------------------------------------------------------------------
# Temperature model (the distance-dependent connection probability that
# Sec. 2.1 sets aside).  Pair {i, j} is an edge iff its coin u = a 2^-53
# (a = temp_coin(seed, i, j)) is below p(d) = 1 / (1 + e^{(d - R)/(2T)}).
# --------------------------------------------------------------------------

def temp_coin(seed: int, i: int, j: int) -> int:
    """a = k + 1 in [1, 2^53] for pair {i, j}: u = a / 2^53."""
    return int(_load().orc_temp_coin(seed & 0xFFFFFFFFFFFFFFFF, int(i), int(j)))


def temp_is_edge(ri, ti, rj, tj, R, T, a):
    """Exact decision of u = a 2^-53 < p(d): (edge, quad_fallbacks, ties)."""
    st = np.zeros(2, dtype=np.int64)
    e = _load().orc_temp_is_edge(ri, ti, rj, tj, R, T, int(a), _p(st, C.c_int64))
    return bool(e), int(st[0]), int(st[1])


def temp_is_edge_quad(ri, ti, rj, tj, R, T, a):
    return bool(_load().orc_temp_is_edge_quad(ri, ti, rj, tj, R, T, int(a)))


def temp_csr(r, theta, R, T, seed, nthreads: int = 0):
    """Every pair tested once with its coin; symmetric CSR with ascending
    rows (int64 row_ptr, int32 col) and (quad_fallbacks, ties)."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = r.shape[0]
    cap = max(1 << 16, 8 * n)
    while True:
        ei = np.empty(cap, dtype=np.int64)
        ej = np.empty(cap, dtype=np.int64)
        st = np.zeros(2, dtype=np.int64)
        m = lib.orc_temp_edges(n, _p(r, C.c_double), _p(theta, C.c_double), R, T,
                               seed & 0xFFFFFFFFFFFFFFFF, _p(ei, C.c_int64), _p(ej, C.c_int64),
                               cap, nthreads, _p(st, C.c_int64))
        if m <= cap:
            break
        cap = int(m)
    src = np.concatenate([ei[:m], ej[:m]])
    dst = np.concatenate([ej[:m], ei[:m]])
    order = np.lexsort((dst, src))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return row_ptr, dst[order].astype(np.int32), int(st[0]), int(st[1])


def temp_rows(r, theta, R, T, seed, which, nthreads: int = 0):
    """Ascending neighbour lists of the vertices in ``which`` under the
    temperature model: (ptr, col, quad_fallbacks, ties)."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    which = np.ascontiguousarray(which, dtype=np.int64)
    n = r.shape[0]
    cap = 1 << 16
    while True:
        ptr = np.zeros(which.shape[0] + 1, dtype=np.int64)
        col = np.empty(cap, dtype=np.int32)
        st = np.zeros(2, dtype=np.int64)
        tot = lib.orc_temp_rows(n, _p(r, C.c_double), _p(theta, C.c_double), R, T,
                                seed & 0xFFFFFFFFFFFFFFFF, _p(which, C.c_int64), which.shape[0],
                                _p(ptr, C.c_int64), _p(col, C.c_int32), cap, nthreads, _p(st, C.c_int64))
        if tot >= 0:
            return ptr, col[:tot].copy(), int(st[0]), int(st[1])
        cap = int(ptr[-1]) + 1


# --------------------------------------------------------------------------
# Dynamic model (vertex movement, Sec. 5): after a batch of moves the graph
# is, by definition, the threshold graph of the moved points, so the oracle
# applies the moves and regenerates by brute force.
# --------------------------------------------------------------------------

def apply_moves(r, theta, ids, r_new, theta_new):
    """The points after the moves (new arrays)."""
    r = np.array(r, dtype=np.float64, copy=True)
    theta = np.array(theta, dtype=np.float64, copy=True)
    ids = np.asarray(ids, dtype=np.int64)
    r[ids] = np.asarray(r_new, dtype=np.float64)
    theta[ids] = np.asarray(theta_new, dtype=np.float64)
    return r, theta
