"""Oracle for displacement-based probing of Tr(P A^{-1}) (arXiv:2106.01275).

TEST INFRASTRUCTURE ONLY.  A plain, slow FP64 CPU implementation of what the
GPU library computes, used by the test suite, the smoke check and the CPU
baseline of the benchmark -- never by the library itself.  It shares no code
with the GPU library: the C part (oracle.c) is compiled here with gcc and
loaded through ctypes; lower bounds and the tile policy are plain Python
(bounds.py).

Every function takes and returns numpy arrays.  Complex vectors are
complex128 arrays of shape [N, nc] (or [nrhs, N, nc]); links are complex128
[4, N, nc, nc] (None = free field, U = 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

NATURAL, REDBLACK, BEST = 0, 1, 2
REAL_Z2, Z2_COMPLEX, Z4 = 0, 1, 2


def build() -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, FP64, -O2)."""
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        vp = ctypes.c_void_p
        L.or_stencil.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64]
        L.or_stencil.restype = ctypes.c_int
        L.or_order.argtypes = [i32p, ctypes.c_int32, i64p]
        L.or_color.argtypes = [i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, i32p]
        L.or_color.restype = ctypes.c_int
        L.or_color_multi.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, i32p]
        L.or_color_multi.restype = ctypes.c_int
        L.or_color_nested.argtypes = [i32p, ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int32,
                                      ctypes.c_int32, i32p, i32p]
        L.or_color_nested.restype = ctypes.c_int
        L.or_mix64.argtypes = [ctypes.c_uint64]
        L.or_mix64.restype = ctypes.c_uint64
        L.or_probe.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_uint64, ctypes.c_int64,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               f64p]
        L.or_apply.argtypes = [i32p, ctypes.c_int32, ctypes.c_double, vp, f64p, f64p]
        L.or_cg.argtypes = [i32p, ctypes.c_int32, ctypes.c_double, vp, f64p, f64p,
                            ctypes.c_double, ctypes.c_int32, vp]
        L.or_cg.restype = ctypes.c_int
        L.or_cg_many.argtypes = [i32p, ctypes.c_int32, ctypes.c_double, vp, ctypes.c_int64,
                                 f64p, f64p, ctypes.c_double, ctypes.c_int32, i32p, vp]
        L.or_trace.argtypes = [i32p, ctypes.c_int32, ctypes.c_double, vp, ctypes.c_int32, i32p,
                               ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                               f64p, f64p, vp, vp]
        L.or_trace.restype = ctypes.c_int
        L.or_trace_grad.argtypes = [i32p, ctypes.c_int32, ctypes.c_double, vp, ctypes.c_int32,
                                    i32p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_int32, f64p, f64p, vp, vp]
        L.or_trace_grad.restype = ctypes.c_int
        _lib = L
    return _lib


def _dims(dims) -> np.ndarray:
    d = np.ones(4, dtype=np.int32)
    dims = list(dims)
    d[: len(dims)] = dims
    return d


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _links(links, N, nc):
    if links is None:
        return None
    a = np.ascontiguousarray(links, dtype=np.complex128)
    assert a.shape == (4, N, nc, nc), a.shape
    return a


# ----------------------------------------------------------------- geometry


def volume(dims) -> int:
    return int(np.prod(_dims(dims), dtype=np.int64))


def stencil(p: int, k: int, d: int = 4) -> np.ndarray:
    """Offsets of N(0,p,k) (Sec. 3, eq. (6)), shape [S, 4]."""
    n = lib().or_stencil(p, k, d, None, 0)
    out = np.zeros((max(n, 1), 4), dtype=np.int32)
    lib().or_stencil(p, k, d, _ptr(out), n)
    return out[:n]


def order(dims, kind: int) -> np.ndarray:
    D = _dims(dims)
    out = np.zeros(volume(D), dtype=np.int64)
    lib().or_order(D, kind, out)
    return out


# ----------------------------------------------------------------- colouring


def coloring(dims, p: int, k: int, order: int = NATURAL, d: int = 4):
    """Greedy displaced distance-k colouring.  BEST = the order (natural,
    red-black) with fewer colours, ties to natural (Sec. 4.1).
    Returns (colors int32[N], ncolors, order used)."""
    D = _dims(dims)
    if order == BEST:
        cn, nn, _ = coloring(dims, p, k, NATURAL, d)
        cr, nr, _ = coloring(dims, p, k, REDBLACK, d)
        return (cn, nn, NATURAL) if nn <= nr else (cr, nr, REDBLACK)
    col = np.zeros(volume(D), dtype=np.int32)
    n = lib().or_color(D, d, p, k, order, col)
    return col, n, order


def coloring_multi(dims, ps, k: int, order: int = NATURAL, d: int = 4):
    """Greedy colouring of N(x, [p_1..p_n], k), the union of the displaced
    neighbourhoods (Sec. 3.4).  Returns (colors int32[N], ncolors)."""
    D = _dims(dims)
    ps = np.ascontiguousarray(ps, dtype=np.int32)
    col = np.zeros(volume(D), dtype=np.int32)
    n = lib().or_color_multi(D, d, ps, len(ps), k, order, col)
    return col, n


def coloring_nested(dims, p: int, ks, order: int = NATURAL, d: int = 4):
    """Nested displaced colourings for increasing distances ks.
    Returns (colors int32[nlev, N], ncolors int32[nlev])."""
    D = _dims(dims)
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    col = np.zeros((len(ks), volume(D)), dtype=np.int32)
    nc = np.zeros(len(ks), dtype=np.int32)
    lib().or_color_nested(D, d, p, ks, len(ks), order, col, nc)
    return col, nc


# ----------------------------------------------------------------- noise & probes


def mix64(z: int) -> int:
    return int(lib().or_mix64(ctypes.c_uint64(z & (2 ** 64 - 1))))


def probe(dims, nc, colors, seed, s, c, a, dilute, kind) -> np.ndarray:
    D = _dims(dims)
    out = np.zeros(volume(D) * nc * 2, dtype=np.float64)
    lib().or_probe(D, nc, np.ascontiguousarray(colors, dtype=np.int32), seed, s, c, a,
                   int(bool(dilute)), kind, out)
    return out.view(np.complex128).reshape(volume(D), nc)


def probes(dims, nc, colors, ncolors, seed, sample0, nsamples, kind, dilute) -> np.ndarray:
    """All probing vectors of samples [sample0, sample0+nsamples), RHS order
    j = ((s - sample0) * ncolors + c) * ndil + a.  Shape [nrhs, N, nc]."""
    ndil = nc if dilute else 1
    out = []
    for s in range(sample0, sample0 + nsamples):
        for c in range(ncolors):
            for a in range(ndil):
                out.append(probe(dims, nc, colors, seed, s, c, a, dilute, kind))
    return np.stack(out)


# ----------------------------------------------------------------- operator & solves


def apply(dims, nc, m2, links, v) -> np.ndarray:
    D = _dims(dims)
    N = volume(D)
    vin = np.ascontiguousarray(v, dtype=np.complex128).reshape(N * nc)
    out = np.zeros(N * nc, dtype=np.complex128)
    L = _links(links, N, nc)
    lib().or_apply(D, nc, m2, _ptr(L), vin.view(np.float64), out.view(np.float64))
    return out.reshape(N, nc)


def dense(dims, nc, m2, links) -> np.ndarray:
    """The operator as a dense (N*nc)^2 matrix, column by column."""
    N = volume(dims)
    n = N * nc
    A = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        A[:, j] = apply(dims, nc, m2, links, e).reshape(n)
    return A


def cg(dims, nc, m2, links, b, tol=1e-12, maxit=100000):
    """Returns (x, iterations (-1 breakdown, -2 no convergence), true rel. residual)."""
    D = _dims(dims)
    N = volume(D)
    bb = np.ascontiguousarray(b, dtype=np.complex128).reshape(N * nc)
    x = np.zeros(N * nc, dtype=np.complex128)
    rr = ctypes.c_double(0.0)
    L = _links(links, N, nc)
    it = lib().or_cg(D, nc, m2, _ptr(L), bb.view(np.float64), x.view(np.float64), tol, maxit,
                     ctypes.byref(rr))
    return x.reshape(N, nc), it, rr.value


def cg_many(dims, nc, m2, links, B, tol=1e-12, maxit=100000):
    """Independent solves for B [nrhs, N, nc]; returns (X, iters[nrhs], relres[nrhs])."""
    D = _dims(dims)
    N = volume(D)
    B = np.ascontiguousarray(B, dtype=np.complex128).reshape(-1, N * nc)
    X = np.zeros_like(B)
    it = np.zeros(B.shape[0], dtype=np.int32)
    rel = np.zeros(B.shape[0], dtype=np.float64)
    L = _links(links, N, nc)
    lib().or_cg_many(D, nc, m2, _ptr(L), B.shape[0], B.view(np.float64), X.view(np.float64),
                     tol, maxit, it, _ptr(rel))
    return X.reshape(-1, N, nc), it, rel


def contractions(dims, nc, V, X, p) -> np.ndarray:
    """t_j = sum_x sum_b conj(v_j(x, b)) x_j(x + p e0, b) for V, X
    [nrhs, N, nc] (Sec. 3: the displaced contraction z^H P x with
    (P x)(x) = x(x + p e0)); unnormalised, one complex value per right-hand
    side.  A numpy restatement of the definition, beside the C one inside
    trace(), for contractions of solutions the caller already has."""
    D = [int(v) for v in _dims(dims)]
    Vs = np.asarray(V, dtype=np.complex128).reshape(-1, *D, nc)
    Xs = np.asarray(X, dtype=np.complex128).reshape(-1, *D, nc)
    Xp = np.roll(Xs, -int(p), axis=1)  # Xp[:, x0] = X[:, x0 + p]
    return np.sum(np.conj(Vs) * Xp, axis=tuple(range(1, Vs.ndim)))


# ----------------------------------------------------------------- estimator


def trace(dims, nc, m2, links, p, colors, ncolors, seed, sample0, nsamples, kind, dilute,
          tol=1e-12, maxit=100000):
    """Probed estimate of Tr(P A^{-1}).  Returns a dict with T (complex),
    stderr, per-sample values T_s, per-RHS contractions t_j and iterations."""
    D = _dims(dims)
    N = volume(D)
    ndil = nc if dilute else 1
    nrhs = nsamples * ncolors * ndil
    out = np.zeros(3)
    per = np.zeros(2 * nsamples)
    tj = np.zeros(2 * nrhs)
    its = np.zeros(nrhs, dtype=np.int32)
    L = _links(links, N, nc)
    st = lib().or_trace(D, nc, m2, _ptr(L), p, np.ascontiguousarray(colors, dtype=np.int32),
                        ncolors, seed, sample0, nsamples, kind, int(bool(dilute)), tol, maxit,
                        out, per, _ptr(tj), _ptr(its))
    if st != 0:
        raise RuntimeError("oracle CG did not converge")
    return {"T": complex(out[0], out[1]), "stderr": out[2],
            "per_sample": per.view(np.complex128).copy(), "tj": tj.view(np.complex128).copy(),
            "iters": its}


def trace_grad(dims, nc, m2, links, p, colors, ncolors, seed, sample0, nsamples, kind, dilute,
               tol=1e-12, maxit=100000):
    """Adjoint gradient of the probed estimate.  Returns (T, dT/dm2,
    dT/dU [4,N,nc,nc], dT/dUbar [4,N,nc,nc]) as complex values/arrays."""
    D = _dims(dims)
    N = volume(D)
    out = np.zeros(3)
    g = np.zeros(2)
    dU = np.zeros((4, N, nc, nc), dtype=np.complex128)
    dUb = np.zeros((4, N, nc, nc), dtype=np.complex128)
    L = _links(links, N, nc)
    st = lib().or_trace_grad(D, nc, m2, _ptr(L), p, np.ascontiguousarray(colors, dtype=np.int32),
                             ncolors, seed, sample0, nsamples, kind, int(bool(dilute)), tol,
                             maxit, out, g, _ptr(dU), _ptr(dUb))
    if st != 0:
        raise RuntimeError("oracle CG did not converge")
    return complex(out[0], out[1]), complex(g[0], g[1]), dU, dUb


def trace_levels(dims, nc, m2, links, p, colors, ncolors, seed, sample0, nsamples, kind, dilute, tol=1e-12):
    """Every level of a nested colouring from the solves of the finest one
    (Sec. 2.3).  With one noise vector per sample for all levels, the probe of
    a class is the sum of the probes of its sub-classes; by linearity the
    level-l estimate is then the sum over the finest probes v_j of
    v_{parent_l(j)}^H P A^{-1} v_j.  colors [L][N] are the levels, coarse to
    fine (the last one is solved), ncolors their colour counts.  Returns one
    dict per level (in the order given) with T, the per-sample values T_s and
    the per-solution terms t_j."""
    colors = [np.asarray(c, dtype=np.int32) for c in colors]
    fine, nfine = colors[-1], int(ncolors[-1])
    ndil = nc if dilute else 1
    V = probes(dims, nc, fine, nfine, seed, sample0, nsamples, kind, dilute)
    X, _, _ = cg_many(dims, nc, m2, links, V, tol=tol)
    out = []
    for col in colors:
        parent = {}
        for x in range(len(fine)):
            parent[int(fine[x])] = int(col[x])
        tj = np.zeros(len(V), dtype=np.complex128)
        j = 0
        for s in range(sample0, sample0 + nsamples):
            for c in range(nfine):
                for a in range(ndil):
                    vp = probe(dims, nc, col, seed, s, parent[c], a, dilute, kind) if c in parent else 0 * V[j]
                    tj[j] = np.vdot(vp, shift(dims, X[j], p))
                    j += 1
        Ts = noise_norm(kind) * tj.reshape(nsamples, -1).sum(axis=1)
        out.append({"T": complex(Ts.mean()), "per_sample": Ts, "tj": tj})
    return out


def noise_norm(kind: int) -> float:
    return 0.5 if kind == Z2_COMPLEX else 1.0


# ----------------------------------------------------------------- deflation (Sec. Deflation)


def lowest_eigenpairs(dims, nc, m2, links, nvec):
    """The nvec smallest eigenvalues of the Hermitian operator (ascending) and
    orthonormal eigenvectors [nvec, N, nc], from the dense matrix (numpy eigh).
    Small lattices only."""
    N = volume(dims)
    w, V = np.linalg.eigh(dense(dims, nc, m2, links))
    return w[:nvec], np.ascontiguousarray(V[:, :nvec].T).reshape(nvec, N, nc)


def shift(dims, v, p):
    """(P v)(x) = v(x + p e0) for v [N, nc] (dim 0 slowest)."""
    D = [int(d) for d in _dims(dims)]
    return np.roll(np.asarray(v).reshape(D + [-1]), -p, axis=0).reshape(np.shape(v))


def trace_deflated(dims, nc, m2, links, p, colors, ncolors, seed, sample0, nsamples, kind, dilute, V):
    """Deflated probed estimate of Tr(P A^{-1}) (Sec. Deflation).

    With the basis V [k, N, nc] (any full-rank set), M = V^H A V and the
    oblique projector Q = A V M^{-1} V^H, the trace splits as
    Tr(P A^{-1} Q) + Tr(P A^{-1} (I - Q)).  Since A^{-1} Q = V M^{-1} V^H the
    first term is evaluated exactly; the second is estimated with the probes,
    t_j = z_j^H P A^{-1} (I - Q) z_j (dense solves).  Per sample
    T_s = T_defl + norm * sum_j t_j.  Small lattices only."""
    N = volume(dims)
    n = N * nc
    A = dense(dims, nc, m2, links)
    Vm = np.asarray(V, dtype=np.complex128).reshape(-1, n).T          # n x k
    AV = A @ Vm
    Minv = np.linalg.inv(Vm.conj().T @ AV)
    # Tr(P V M^{-1} V^H) = sum_x sum_b (V M^{-1} V^H)[(x + p e0, b), (x, b)]
    Dm = Vm @ Minv @ Vm.conj().T
    rows = shift(dims, np.arange(n).reshape(N, nc), p).reshape(n)   # index of (x + p e0, b)
    T_defl = complex(np.sum(Dm[rows, np.arange(n)]))
    Z = probes(dims, nc, colors, ncolors, seed, sample0, nsamples, kind, dilute).reshape(-1, n)
    B = Z.T - AV @ (Minv @ (Vm.conj().T @ Z.T))                     # (I - Q) z, columns
    X = np.linalg.solve(A, B)
    tj = np.array([np.vdot(Z[j], shift(dims, X[:, j].reshape(N, nc), p).reshape(n))
                   for j in range(Z.shape[0])])
    norm = noise_norm(kind)
    per = Z.shape[0] // nsamples
    Ts = T_defl + norm * tj.reshape(nsamples, per).sum(axis=1)
    T = complex(Ts.mean())
    stderr = float(np.sqrt(np.sum(np.abs(Ts - T) ** 2) / (nsamples - 1) / nsamples)) if nsamples > 1 else float("nan")
    return {"T": T, "T_defl": T_defl, "per_sample": Ts, "tj": tj, "stderr": stderr}
