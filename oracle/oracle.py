"""Python access to the CPU oracle (test infrastructure only).

The oracle lists every k-clique explicitly and runs synchronous Frank-Wolfe on
the convex program CP(G) (paper Sec. 2, Algorithm 1), then extracts the best
prefix by k-clique density (Algorithm 2's final steps).  It is the yardstick of
the GPU path and is loaded only by tests, the smoke check and the benchmark's
CPU-baseline leg.  It imports nothing from the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kdss_oracle.c")
LIB = os.path.join(HERE, "libkdss_oracle.so")


class Result(C.Structure):
    _fields_ = [("c_k_lo", C.c_uint64), ("c_k_hi", C.c_uint64), ("T", C.c_uint32),
                ("size", C.c_uint32), ("dens_num", C.c_uint64), ("ub_num_lo", C.c_uint64),
                ("ub_num_hi", C.c_uint64), ("enum_seconds", C.c_double),
                ("iter_seconds", C.c_double), ("extract_seconds", C.c_double),
                ("threads", C.c_int), ("streamed", C.c_int)]


class TraceRow(C.Structure):
    _fields_ = [("t", C.c_uint32), ("size", C.c_uint32), ("dens_num", C.c_uint64),
                ("ub_num_lo", C.c_uint64), ("ub_num_hi", C.c_uint64)]


def build(force: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle (or a copy of its source) with gcc: plain C, OpenMP."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, src])
        os.replace(tmp, out)
    return out


_libs = {}


def lib(path: str | None = None):
    """The oracle library at ``path`` (default: the built oracle)."""
    path = path or LIB
    if path not in _libs:
        if path == LIB and not os.path.exists(LIB):
            build()
        L = C.CDLL(path)
        p64 = C.POINTER(C.c_uint64)
        p32 = C.POINTER(C.c_uint32)
        L.kor_validate.argtypes = [C.c_uint32, C.c_uint64, p64, p32]
        L.kor_count.argtypes = [C.c_uint32, p64, p32, C.c_int, C.c_int, p64, p64]
        L.kor_list.argtypes = [C.c_uint32, p64, p32, C.c_int, p32, C.c_uint64, p64]
        L.kor_solve.argtypes = [C.c_uint32, p64, p32, C.c_int, C.c_uint32, p64, C.c_int,
                                C.c_uint64, p64, p64, p32, C.POINTER(Result),
                                C.POINTER(TraceRow)]
        L.kor_credits.argtypes = [C.c_uint32, p64, p32, C.c_int, p64, p64]
        L.kor_threads.argtypes = [C.c_int]
        L.kor_extract.argtypes = [C.c_uint32, p64, p32, C.c_int, p64, C.c_int, p32, p32, p64]
        L.kor_prefix_counts.argtypes = [C.c_uint32, p64, p32, C.c_int, p64, C.c_int, p32, p32, p64, p64]
        L.kor_pb_pair.argtypes = [C.c_uint32, p32, C.c_uint32, C.c_uint32, C.c_int, p64, p64]
        L.kor_pb_run.argtypes = [C.c_uint32, C.c_uint64, p32, p32, p64, p32, C.c_int, C.c_uint32, C.c_int,
                                 p64, C.POINTER(C.c_double)]
        L.kor_color.argtypes = [C.c_uint32, p64, p32, p32]
        L.kor_sample.argtypes = [C.c_uint32, p64, p32, C.c_int, C.c_uint64, p64, p32, C.POINTER(C.c_uint8),
                                 p64, p64]
        L.kor_solve_list.argtypes = [C.c_uint32, p32, C.c_uint64, C.c_int, C.c_uint32, p64, p32, p32, p64]
        _libs[path] = L
    return _libs[path]


def _p64(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64)) if a is not None else None


def _p32(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32)) if a is not None else None


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    cl = np.ascontiguousarray(col, dtype=np.uint32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.uint32)
    return rp, cl


def validate(n, row_ptr, col, libpath=None) -> int:
    rp, cl = _csr(row_ptr, col)
    return lib(libpath).kor_validate(n, int(rp[n]) if rp.size > n else 0, _p64(rp), _p32(cl))


def count(n, row_ptr, col, k, threads=0, libpath=None) -> int:
    rp, cl = _csr(row_ptr, col)
    lo, hi = C.c_uint64(0), C.c_uint64(0)
    err = lib(libpath).kor_count(n, _p64(rp), _p32(cl), k, threads, C.byref(lo), C.byref(hi))
    if err:
        raise RuntimeError(f"kor_count failed: {err}")
    return (hi.value << 64) | lo.value


def list_cliques(n, row_ptr, col, k, libpath=None) -> np.ndarray:
    """All k-cliques as rows of ascending ids (lexicographic order)."""
    c = count(n, row_ptr, col, k, libpath=libpath)
    rp, cl = _csr(row_ptr, col)
    out = np.zeros(max(c, 1) * k, dtype=np.uint32)
    got = C.c_uint64(0)
    err = lib(libpath).kor_list(n, _p64(rp), _p32(cl), k, _p32(out), c, C.byref(got))
    if err:
        raise RuntimeError(f"kor_list failed: {err}")
    return out[: c * k].reshape(c, k)


def credits(n, row_ptr, col, k, r, libpath=None) -> np.ndarray:
    """Frank-Wolfe credits d(u) of one synchronous iteration at loads r."""
    rp, cl = _csr(row_ptr, col)
    rr = np.ascontiguousarray(r, dtype=np.uint64)
    d = np.zeros(max(n, 1), dtype=np.uint64)
    err = lib(libpath).kor_credits(n, _p64(rp), _p32(cl), k, _p64(rr), _p64(d))
    if err:
        raise RuntimeError(f"kor_credits failed: {err}")
    return d[:n]


def solve(n, row_ptr, col, k, T, r0=None, trace=False, threads=0,
          max_store_bytes=8 << 30, libpath=None) -> dict:
    """Synchronous Frank-Wolfe + extraction.  Returns a dict with
    r (uint64 when every load fits, else Python ints), order (uint32[n]),
    size (i*), dens_num (K_{i*}), ub_num (max r_T - r0), T, c_k, timings and,
    when asked, the per-iteration trace."""
    rp, cl = _csr(row_ptr, col)
    nn = max(n, 1)
    r_lo = np.zeros(nn, dtype=np.uint64)
    r_hi = np.zeros(nn, dtype=np.uint64)
    order = np.zeros(nn, dtype=np.uint32)
    r0a = None if r0 is None else np.ascontiguousarray(r0, dtype=np.uint64)
    res = Result()
    rows = (TraceRow * T)() if trace else None
    err = lib(libpath).kor_solve(n, _p64(rp), _p32(cl), k, T, _p64(r0a), threads, max_store_bytes,
                          _p64(r_lo), _p64(r_hi), _p32(order), C.byref(res),
                          C.cast(rows, C.POINTER(TraceRow)) if trace else None)
    if err:
        raise RuntimeError(f"kor_solve failed: {err}")
    if np.any(r_hi[:n]):
        r = [(int(h) << 64) | int(l) for l, h in zip(r_lo[:n], r_hi[:n])]
    else:
        r = r_lo[:n].copy()
    out = dict(r=r, order=order[:n].copy(), size=res.size, dens_num=res.dens_num,
               ub_num=(res.ub_num_hi << 64) | res.ub_num_lo, T=res.T,
               c_k=(res.c_k_hi << 64) | res.c_k_lo, enum_seconds=res.enum_seconds,
               iter_seconds=res.iter_seconds, extract_seconds=res.extract_seconds,
               threads=res.threads, streamed=bool(res.streamed))
    if trace:
        out["trace"] = [dict(t=rw.t, size=rw.size, dens_num=rw.dens_num,
                             ub_num=(rw.ub_num_hi << 64) | rw.ub_num_lo) for rw in rows]
    return out


def extract(n, row_ptr, col, k, r, threads=0, libpath=None) -> dict:
    """The extraction alone at loads r (uint64): order, size i* and K_{i*}."""
    rp, cl = _csr(row_ptr, col)
    rr = np.ascontiguousarray(r, dtype=np.uint64)
    order = np.zeros(max(n, 1), dtype=np.uint32)
    size = C.c_uint32(0)
    dens = np.zeros(1, dtype=np.uint64)
    err = lib(libpath).kor_extract(n, _p64(rp), _p32(cl), k, _p64(rr), threads, _p32(order), C.byref(size),
                                   _p64(dens))
    if err:
        raise RuntimeError(f"kor_extract failed: {err}")
    return dict(order=order[:n], size=size.value, dens_num=int(dens[0]))


def prefix_counts(n, row_ptr, col, k, r, threads=0, libpath=None) -> dict:
    """The extraction at loads r (uint64) with every prefix count:
    K[i - 1] = |C_k(order[0 .. i))| for i = 1..n."""
    rp, cl = _csr(row_ptr, col)
    rr = np.ascontiguousarray(r, dtype=np.uint64)
    order = np.zeros(max(n, 1), dtype=np.uint32)
    K = np.zeros(max(n, 1), dtype=np.uint64)
    size = C.c_uint32(0)
    dens = np.zeros(1, dtype=np.uint64)
    err = lib(libpath).kor_prefix_counts(n, _p64(rp), _p32(cl), k, _p64(rr), threads, _p32(order),
                                         C.byref(size), _p64(dens), _p64(K))
    if err:
        raise RuntimeError(f"kor_prefix_counts failed: {err}")
    return dict(order=order[:n], size=size.value, dens_num=int(dens[0]), K=K[:n])


def pb_pair(n, members, h, p, k, r, libpath=None) -> np.ndarray:
    """PBUpdate (Algorithm 3) of one pair at loads r: the increments of its nodes."""
    mem = np.ascontiguousarray(members, dtype=np.uint32)
    rr = np.ascontiguousarray(r, dtype=np.uint64)
    d = np.zeros(max(n, 1), dtype=np.uint64)
    err = lib(libpath).kor_pb_pair(n, _p32(mem), h, p, k, _p64(rr), _p64(d))
    if err:
        raise RuntimeError(f"kor_pb_pair failed: {err}")
    return d[:n]


def pb_run(n, h, p, members, k, T, synchronous, r0=None, libpath=None) -> dict:
    """T iterations of PBUpdate over the pairs (h[q], p[q], members flattened,
    hold nodes first), sequential (the paper's loop) or synchronous."""
    hh = np.ascontiguousarray(h, dtype=np.uint32)
    pp = np.ascontiguousarray(p, dtype=np.uint32)
    mem = np.ascontiguousarray(members, dtype=np.uint32)
    off = np.zeros(len(hh) + 1, dtype=np.uint64)
    np.cumsum(hh.astype(np.uint64) + pp.astype(np.uint64), out=off[1:])
    r = np.zeros(max(n, 1), dtype=np.uint64)
    if r0 is not None:
        r[:n] = np.asarray(r0, dtype=np.uint64)
    secs = C.c_double(0.0)
    err = lib(libpath).kor_pb_run(n, len(hh), _p32(hh), _p32(pp), _p64(off), _p32(mem), k, T,
                                  1 if synchronous else 0, _p64(r), C.byref(secs))
    if err:
        raise RuntimeError(f"kor_pb_run failed: {err}")
    return dict(r=r[:n], seconds=secs.value)


def top_bound(r, r0, T, k):
    """A certified bound on rho* = max_S |C_k(S)| / |S| from Frank-Wolfe loads:
    every S of s nodes has |C_k(S)| <= (sum over S of (r - r0)) / T (the
    cliques inside S put their weight inside S) and |C_k(S)| <= C(s, k), so
    rho* <= max_s min(A_s, T C(s, k)) / (T s), A_s = the s largest (r - r0)."""
    from fractions import Fraction
    import math
    base = [0] * len(r) if r0 is None else [int(x) for x in r0]
    vals = sorted((int(a) - b for a, b in zip(r, base)), reverse=True)
    best, A = Fraction(0), 0
    for s, x in enumerate(vals, 1):
        A += x
        best = max(best, Fraction(min(A, T * math.comb(s, k)), T * s))
    return best


def certified(dens_num, size, bound, n):
    """Distinct densities with denominators <= n differ by at least
    1 / (n (n - 1)): a density within that of a bound on rho* is rho*."""
    from fractions import Fraction
    rho = Fraction(dens_num, size) if size else Fraction(0)
    if bound < rho:
        return False
    return n < 2 or bound - rho < Fraction(1, n * (n - 1))


def color(n, row_ptr, col, libpath=None) -> np.ndarray:
    """Greedy colouring, nodes by degree (descending, ties by id)."""
    rp, cl = _csr(row_ptr, col)
    c = np.zeros(max(n, 1), dtype=np.uint32)
    err = lib(libpath).kor_color(n, _p64(rp), _p32(cl), _p32(c))
    if err:
        raise RuntimeError(f"kor_color failed: {err}")
    return c[:n]


def sample(n, row_ptr, col, k, draws, libpath=None) -> dict:
    """k-color path samples (Algorithm 4's first step) from given draws
    (uint64[t, k, 2]): per sample its sorted ids and whether it is a k-clique,
    plus the number of colour-increasing k-node paths."""
    rp, cl = _csr(row_ptr, col)
    d = np.ascontiguousarray(draws, dtype=np.uint64)
    t = d.shape[0] if d.size else 0
    out = np.zeros(max(t * k, 1), dtype=np.uint32)
    valid = np.zeros(max(t, 1), dtype=np.uint8)
    lo = C.c_uint64(0)
    hi = C.c_uint64(0)
    err = lib(libpath).kor_sample(n, _p64(rp), _p32(cl), k, t, _p64(d.reshape(-1)) if t else None, _p32(out),
                                  valid.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(lo), C.byref(hi))
    if err:
        raise RuntimeError(f"kor_sample failed: {err}")
    return dict(cliques=out[: t * k].reshape(t, k), valid=valid[:t].astype(bool),
                paths=(hi.value << 64) | lo.value)


def solve_list(n, cliques, k, T, libpath=None) -> dict:
    """Synchronous Frank-Wolfe and the extraction over a given clique list."""
    cl = np.ascontiguousarray(cliques, dtype=np.uint32).reshape(-1)
    ncl = cl.size // k
    r = np.zeros(max(n, 1), dtype=np.uint64)
    order = np.zeros(max(n, 1), dtype=np.uint32)
    size = C.c_uint32(0)
    dens = np.zeros(1, dtype=np.uint64)
    err = lib(libpath).kor_solve_list(n, _p32(cl) if ncl else None, ncl, k, T, _p64(r), _p32(order),
                                      C.byref(size), _p64(dens))
    if err:
        raise RuntimeError(f"kor_solve_list failed: {err}")
    return dict(r=r[:n], order=order[:n], size=size.value, dens_num=int(dens[0]))
