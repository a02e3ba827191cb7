"""Python binding of libdprobe, the gfx950 library for displacement-based
probing of Tr(P A^{-1}) (arXiv:2106.01275).

Argument marshalling only: every step of the method runs in the library's
HIP kernels (or, for the colouring, its host code).  PyTorch provides device
memory and streams.  The names follow the C ABI in include/dp.h:

    build_coloring, build_coloring_multi, tile_shape, build_coloring_tiled,
    clearance, make_probes, solve_batch, trace_estimate, trace_multi,
    trace_grad, apply (the operator, for verification)

plus ProbedTrace, a torch.autograd.Function over trace_estimate/trace_grad.
The library must be built (python -m paper_2106_01275_amd.build); importing
this module never falls back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdprobe.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, EUNSUPPORTED = range(7)
ORDER = {"natural": 0, "redblack": 1, "best": 2}
NOISE = {"real_z2": 0, "z2_complex": 1, "z4": 2}
PREC = {"f64": 0, "f32": 1, "bf16": 2}
NOISE_NORM = {"real_z2": 1.0, "z2_complex": 0.5, "z4": 1.0}

_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ENOCONV", 5: "EBREAKDOWN", 6: "EUNSUPPORTED"}


class DPError(RuntimeError):
    def __init__(self, status, msg, result=None):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.result = result


class ProbeSpec(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("nc", ctypes.c_int32), ("colors_dev", ctypes.c_void_p),
                ("ncolors", ctypes.c_int32), ("seed", ctypes.c_uint64), ("sample0", ctypes.c_int32),
                ("nsamples", ctypes.c_int32), ("noise", ctypes.c_int32), ("dilute", ctypes.c_int32)]


class Operator(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("nc", ctypes.c_int32), ("m2", ctypes.c_double),
                ("links", ctypes.c_void_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("rhs_block", ctypes.c_int32), ("reliable_delta", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("profile", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("nrhs", ctypes.c_int64), ("rhs_iters", ctypes.c_int64), ("max_iters", ctypes.c_int32),
                ("nconverged", ctypes.c_int32), ("nbreakdown", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("max_true_resid", ctypes.c_double),
                ("rhs_block", ctypes.c_int32), ("stencil_launches", ctypes.c_int32),
                ("stencil_ms", ctypes.c_double), ("stencil_bytes", ctypes.c_double),
                ("seconds", ctypes.c_double), ("stencil_bytes_all", ctypes.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TraceResult(ctypes.Structure):
    _fields_ = [("tr", ctypes.c_double * 2), ("stderr_", ctypes.c_double),
                ("per_sample", ctypes.c_void_p), ("per_rhs", ctypes.c_void_p), ("solve", SolveStats)]


class EigOpts(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("max_outer", ctypes.c_int32), ("tol", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


EXPORTS = ["dp_create", "dp_destroy", "dp_last_error", "dp_build_coloring", "dp_build_coloring_multi",
           "dp_tile_shape", "dp_build_coloring_tiled", "dp_clearance", "dp_make_probes", "dp_solve_batch",
           "dp_trace_estimate", "dp_trace_multi", "dp_trace_levels", "dp_trace_grad", "dp_apply",
           "dp_solve_noalloc", "dp_deflation_create",
           "dp_deflation_info", "dp_deflation_vectors", "dp_trace_deflated", "dp_deflation_destroy"]

_lib = None


def lib():
    """Loads libdprobe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2106_01275_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.dp_create.argtypes = [ctypes.POINTER(vp), i32]
        L.dp_destroy.argtypes = [vp]
        L.dp_destroy.restype = None
        L.dp_last_error.argtypes = [vp]
        L.dp_last_error.restype = ctypes.c_char_p
        L.dp_build_coloring.argtypes = [vp, i32, vp, i32, i32, vp, vp, vp]
        L.dp_build_coloring_multi.argtypes = [vp, vp, i32, vp, i32, i32, vp, vp, vp]
        L.dp_tile_shape.argtypes = [vp, i32, i32, vp]
        L.dp_build_coloring_tiled.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.dp_clearance.argtypes = [vp, vp, i32, i32, vp]
        L.dp_make_probes.argtypes = [vp, ctypes.POINTER(ProbeSpec), i64, i64, vp, vp]
        L.dp_solve_batch.argtypes = [vp, i32, ctypes.POINTER(Operator), vp, vp, vp,
                                     ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]
        L.dp_trace_estimate.argtypes = [vp, i32, ctypes.POINTER(Operator), vp, ctypes.POINTER(ProbeSpec),
                                        ctypes.POINTER(SolveOpts), ctypes.POINTER(TraceResult), vp]
        L.dp_trace_multi.argtypes = [vp, ctypes.POINTER(Operator), vp, i32, ctypes.POINTER(ProbeSpec),
                                     ctypes.POINTER(SolveOpts), ctypes.POINTER(TraceResult), vp]
        L.dp_trace_levels.argtypes = [vp, ctypes.POINTER(Operator), i32, ctypes.POINTER(ProbeSpec), i32, vp, vp,
                                      ctypes.POINTER(SolveOpts), ctypes.POINTER(TraceResult), vp]
        L.dp_trace_grad.argtypes = [vp, ctypes.POINTER(Operator), i32, ctypes.POINTER(ProbeSpec),
                                    ctypes.POINTER(SolveOpts), ctypes.POINTER(TraceResult), vp, vp, vp, vp]
        L.dp_apply.argtypes = [vp, ctypes.POINTER(Operator), i32, vp, vp, i64, vp]
        L.dp_solve_noalloc.argtypes = [vp, ctypes.POINTER(Operator), vp, vp, i64, ctypes.POINTER(SolveOpts),
                                       ctypes.POINTER(SolveStats), vp]
        L.dp_deflation_create.argtypes = [vp, ctypes.POINTER(Operator), i32, ctypes.POINTER(EigOpts),
                                          ctypes.POINTER(vp), vp]
        L.dp_deflation_info.argtypes = [vp, vp, vp, vp, vp]
        L.dp_deflation_vectors.argtypes = [vp, vp, vp, vp]
        L.dp_trace_deflated.argtypes = [vp, ctypes.POINTER(Operator), vp, i32, ctypes.POINTER(ProbeSpec),
                                        ctypes.POINTER(SolveOpts), ctypes.POINTER(TraceResult), vp, vp]
        L.dp_deflation_destroy.argtypes = [vp]
        L.dp_deflation_destroy.restype = None
        for name in ("dp_create", "dp_build_coloring", "dp_build_coloring_multi", "dp_tile_shape",
                     "dp_build_coloring_tiled", "dp_clearance", "dp_make_probes", "dp_solve_batch",
                     "dp_trace_estimate", "dp_trace_multi", "dp_trace_levels", "dp_trace_grad", "dp_apply",
                     "dp_solve_noalloc", "dp_deflation_create", "dp_deflation_info", "dp_deflation_vectors", "dp_trace_deflated"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _dims4(dims):
    d = [1, 1, 1, 1]
    d[: len(dims)] = [int(v) for v in dims]
    return d


def build_coloring(dims, p, ks, order="natural"):
    """Greedy displaced colouring (host).  ks: one distance or an increasing
    list (nested levels).  Returns (colors int32[nlev, N] or [N], ncolors,
    order used)."""
    flat = np.isscalar(ks)
    ks = _i32([ks] if flat else list(ks))
    d = _i32(_dims4(dims))
    N = int(np.prod(d))
    col = np.zeros((len(ks), N), dtype=np.int32)
    nc = np.zeros(len(ks), dtype=np.int32)
    used = np.zeros(1, dtype=np.int32)
    st = lib().dp_build_coloring(d.ctypes.data, int(p), ks.ctypes.data, len(ks), ORDER[order],
                                 col.ctypes.data, nc.ctypes.data, used.ctypes.data)
    if st != OK:
        raise DPError(st, lib().dp_last_error(None).decode())
    used_name = {v: k for k, v in ORDER.items()}[int(used[0])]
    if flat:
        return col[0], int(nc[0]), used_name
    return col, nc, used_name


def build_coloring_multi(dims, disps, ks, order="natural"):
    """Greedy colouring of the union of the displaced neighbourhoods of the
    displacements disps (Sec. 3.4).  Same returns as build_coloring."""
    flat = np.isscalar(ks)
    ks = _i32([ks] if flat else list(ks))
    d = _i32(_dims4(dims))
    ds = _i32(list(disps))
    N = int(np.prod(d))
    col = np.zeros((len(ks), N), dtype=np.int32)
    nc = np.zeros(len(ks), dtype=np.int32)
    used = np.zeros(1, dtype=np.int32)
    st = lib().dp_build_coloring_multi(d.ctypes.data, ds.ctypes.data, len(ds), ks.ctypes.data, len(ks),
                                       ORDER[order], col.ctypes.data, nc.ctypes.data, used.ctypes.data)
    if st != OK:
        raise DPError(st, lib().dp_last_error(None).decode())
    used_name = {v: k for k, v in ORDER.items()}[int(used[0])]
    if flat:
        return col[0], int(nc[0]), used_name
    return col, nc, used_name


def tile_shape(dims, p, k):
    """Tile of the (p, k) colouring (Sec. 3.5), a tuple of 4 extents."""
    d = _i32(_dims4(dims))
    t = np.zeros(4, dtype=np.int32)
    st = lib().dp_tile_shape(d.ctypes.data, int(p), int(k), t.ctypes.data)
    if st != OK:
        raise DPError(st, lib().dp_last_error(None).decode())
    return tuple(int(v) for v in t)


def build_coloring_tiled(dims, p, k, order="natural"):
    """Tiled (p, k) colouring (Sec. 3.5): returns (colors int32[N], ncolors,
    order used, tile).  DP_COLOR_CACHE (a directory) caches tile colourings."""
    d = _i32(_dims4(dims))
    N = int(np.prod(d))
    col = np.zeros(N, dtype=np.int32)
    nc = np.zeros(1, dtype=np.int32)
    used = np.zeros(1, dtype=np.int32)
    t = np.zeros(4, dtype=np.int32)
    st = lib().dp_build_coloring_tiled(d.ctypes.data, int(p), int(k), ORDER[order], col.ctypes.data,
                                       nc.ctypes.data, used.ctypes.data, t.ctypes.data)
    if st != OK:
        raise DPError(st, lib().dp_last_error(None).decode())
    return col, int(nc[0]), {v: k_ for k_, v in ORDER.items()}[int(used[0])], tuple(int(v) for v in t)


def clearance(dims, colors, p, kmax):
    """Table Clearance (Sec. 4.3): percentage of the sites at distance
    exactly k (k = 0..kmax) from x +- p e0 that share the colour of x,
    averaged over x.  Returns float64[kmax + 1]."""
    d = _i32(_dims4(dims))
    col = _i32(colors)
    out = np.zeros(kmax + 1)
    st = lib().dp_clearance(d.ctypes.data, col.ctypes.data, int(p), int(kmax), out.ctypes.data)
    if st != OK:
        raise DPError(st, lib().dp_last_error(None).decode())
    return out


class Context:
    """A library context bound to one HIP device (the torch device index)."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = device
        h = ctypes.c_void_p()
        st = lib().dp_create(ctypes.byref(h), device)
        if st != OK:
            raise DPError(st, lib().dp_last_error(None).decode())
        self.h = h

    def close(self):
        if self.h:
            lib().dp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _err(self, st, result=None):
        raise DPError(st, lib().dp_last_error(self.h).decode(), result)

    def _cdev(self, t, dtype, numel=None):
        # the kernels trust the sizes: check them here, on the host
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
            raise TypeError(f"expected a contiguous {dtype} tensor on the GPU")
        if (t.device.index or 0) != self.device:
            raise ValueError(f"tensor on cuda:{t.device.index}, context on cuda:{self.device}")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"expected {numel} elements, got {t.numel()} (shape {tuple(t.shape)})")
        return ctypes.c_void_p(t.data_ptr())

    def operator(self, dims, nc, m2, links=None):
        """links: complex128 cuda tensor [4, N, nc, nc] or None (U = 1)."""
        op = Operator()
        op.dims[:] = _dims4(dims)
        op.nc = nc
        op.m2 = float(m2)
        N = int(np.prod(list(op.dims)))
        op.links = None if links is None else self._cdev(links, self.torch.complex128, 4 * N * nc * nc).value
        op._keep = links
        return op

    def probe_spec(self, dims, nc, colors_dev, ncolors, seed, sample0, nsamples, noise, dilute):
        ps = ProbeSpec()
        ps.dims[:] = _dims4(dims)
        ps.nc = nc
        ps.colors_dev = self._cdev(colors_dev, self.torch.int32, int(np.prod(list(ps.dims)))).value
        ps.ncolors = int(ncolors)
        ps.seed = int(seed)
        ps.sample0 = int(sample0)
        ps.nsamples = int(nsamples)
        ps.noise = NOISE[noise] if isinstance(noise, str) else int(noise)
        ps.dilute = int(bool(dilute))
        ps._keep = colors_dev
        return ps

    @staticmethod
    def opts(tol=1e-10, max_iter=0, inner="f64", rhs_block=0, reliable_delta=0.0, use_graph=0, profile=0):
        o = SolveOpts()
        o.tol = tol
        o.max_iter = max_iter
        o.inner = PREC[inner] if isinstance(inner, str) else int(inner)
        o.rhs_block = rhs_block
        o.reliable_delta = reliable_delta
        o.use_graph = use_graph
        o.profile = profile
        return o

    # ------------------------------------------------------------ entry points
    def make_probes(self, ps, rhs0, nrhs, out=None):
        torch = self.torch
        N = int(np.prod(list(ps.dims)))
        if out is None:
            out = torch.empty((nrhs, N, ps.nc), dtype=torch.complex128, device=f"cuda:{self.device}")
        st = lib().dp_make_probes(self.h, ctypes.byref(ps), rhs0, nrhs,
                                  self._cdev(out, torch.complex128, nrhs * N * ps.nc), self._stream())
        if st != OK:
            self._err(st)
        return out

    def solve_batch(self, ops, bs, opts, xs=None, check=True):
        """ops: list of Operator; bs: list of complex128 [nrhs, N, nc] tensors."""
        torch = self.torch
        n = len(ops)
        if xs is None:
            xs = [torch.empty_like(b) for b in bs]
        arr_ops = (Operator * n)(*ops)
        if len(bs) != n or len(xs) != n:
            raise ValueError("one right-hand-side and one solution tensor per operator")
        # (an operator with a dimension < 1 is left to the library, which rejects it)
        sizes = [b.shape[0] * int(np.prod(list(op.dims))) * op.nc if min(op.dims) >= 1 else None
                 for b, op in zip(bs, ops)]
        pb = (ctypes.c_void_p * n)(*[self._cdev(b, torch.complex128, m).value for b, m in zip(bs, sizes)])
        px = (ctypes.c_void_p * n)(*[self._cdev(x, torch.complex128, m).value for x, m in zip(xs, sizes)])
        nr = (ctypes.c_int64 * n)(*[b.shape[0] for b in bs])
        stats = (SolveStats * n)()
        st = lib().dp_solve_batch(self.h, n, arr_ops, pb, px, nr, ctypes.byref(opts), stats, self._stream())
        res = (xs, [s.asdict() for s in stats])
        if st != OK and (check or st not in (ENOCONV, EBREAKDOWN)):
            self._err(st, res)
        return res

    def trace_estimate(self, ops, ps, p, opts, check=True):
        """ops, ps, p: lists (one entry per instance).  Returns a list of dicts."""
        n = len(ops)
        arr_ops = (Operator * n)(*ops)
        arr_ps = (ProbeSpec * n)(*ps)
        arr_p = (ctypes.c_int32 * n)(*[int(v) for v in p])
        res = (TraceResult * n)()
        bufs = []
        for i in range(n):
            ndil = ps[i].nc if ps[i].dilute else 1
            nrhs = ps[i].nsamples * ps[i].ncolors * ndil
            per_s = np.zeros(2 * ps[i].nsamples)
            per_r = np.zeros(2 * nrhs)
            bufs.append((per_s, per_r))
            res[i].per_sample = per_s.ctypes.data
            res[i].per_rhs = per_r.ctypes.data
        st = lib().dp_trace_estimate(self.h, n, arr_ops, arr_p, arr_ps, ctypes.byref(opts), res,
                                     self._stream())
        out = []
        for i in range(n):
            out.append({"T": complex(res[i].tr[0], res[i].tr[1]), "stderr": res[i].stderr_,
                        "per_sample": bufs[i][0].view(np.complex128).copy(),
                        "tj": bufs[i][1].view(np.complex128).copy(), "solve": res[i].solve.asdict()})
        if st != OK and (check or st not in (ENOCONV, EBREAKDOWN)):
            self._err(st, out)
        return out

    def trace_multi(self, op, ps, disps, opts, check=True):
        """One probe set solved once, contracted with every displacement in
        disps (any sign).  Returns a list of dicts (one per displacement)."""
        n = len(disps)
        arr_d = (ctypes.c_int32 * n)(*[int(v) for v in disps])
        res = (TraceResult * n)()
        ndil = ps.nc if ps.dilute else 1
        nrhs = ps.nsamples * ps.ncolors * ndil
        bufs = []
        for i in range(n):
            per_s, per_r = np.zeros(2 * ps.nsamples), np.zeros(2 * nrhs)
            bufs.append((per_s, per_r))
            res[i].per_sample = per_s.ctypes.data
            res[i].per_rhs = per_r.ctypes.data
        st = lib().dp_trace_multi(self.h, ctypes.byref(op), arr_d, n, ctypes.byref(ps), ctypes.byref(opts), res,
                                  self._stream())
        out = [{"p": int(disps[i]), "T": complex(res[i].tr[0], res[i].tr[1]), "stderr": res[i].stderr_,
                "per_sample": bufs[i][0].view(np.complex128).copy(), "tj": bufs[i][1].view(np.complex128).copy(),
                "solve": res[i].solve.asdict()} for i in range(n)]
        if st != OK and (check or st not in (ENOCONV, EBREAKDOWN)):
            self._err(st, out)
        return out

    def trace_levels(self, op, ps, p, coarse, opts, check=True):
        """Every level of a nested colouring from the solves of the finest one
        (ps).  coarse: list of (colours, ncolours) of the coarser levels,
        colours an int32 cuda tensor [N] each.  Returns a list of dicts, the
        finest level first, then the coarse levels in the order given."""
        N = int(np.prod(list(ps.dims)))
        n = len(coarse)
        keep = [self._cdev(c, self.torch.int32, N) for c, _ in coarse]
        arr_c = (ctypes.c_void_p * max(n, 1))(*[k.value for k in keep])
        arr_n = (ctypes.c_int32 * max(n, 1))(*[int(m) for _, m in coarse])
        res = (TraceResult * (n + 1))()
        ndil = ps.nc if ps.dilute else 1
        nrhs = ps.nsamples * ps.ncolors * ndil
        bufs = []
        for i in range(n + 1):
            per_s, per_r = np.zeros(2 * ps.nsamples), np.zeros(2 * nrhs)
            bufs.append((per_s, per_r))
            res[i].per_sample = per_s.ctypes.data
            res[i].per_rhs = per_r.ctypes.data
        st = lib().dp_trace_levels(self.h, ctypes.byref(op), int(p), ctypes.byref(ps), n, arr_c, arr_n,
                                   ctypes.byref(opts), res, self._stream())
        out = [{"T": complex(res[i].tr[0], res[i].tr[1]), "stderr": res[i].stderr_,
                "per_sample": bufs[i][0].view(np.complex128).copy(), "tj": bufs[i][1].view(np.complex128).copy(),
                "solve": res[i].solve.asdict()} for i in range(n + 1)]
        if st != OK and (check or st not in (ENOCONV, EBREAKDOWN)):
            self._err(st, out)
        return out

    def trace_grad(self, op, ps, p, opts, want_links=True, check=True):
        """Returns (T, dT/dm2, dT/dU, dT/dUbar, stats); the link gradients are
        complex128 cuda tensors [4, N, nc, nc] (None if want_links is False);
        stats["tj"] holds the per-right-hand-side contractions t_j."""
        torch = self.torch
        N = int(np.prod(list(op.dims)))
        res = TraceResult()
        ndil = ps.nc if ps.dilute else 1
        per_r = np.zeros(2 * ps.nsamples * ps.ncolors * ndil)
        res.per_rhs = per_r.ctypes.data
        g = (ctypes.c_double * 2)()
        dU = dUb = None
        if want_links:
            dU = torch.empty((4, N, op.nc, op.nc), dtype=torch.complex128, device=f"cuda:{self.device}")
            dUb = torch.empty_like(dU)
        st = lib().dp_trace_grad(self.h, ctypes.byref(op), int(p), ctypes.byref(ps), ctypes.byref(opts),
                                 ctypes.byref(res), g,
                                 None if dU is None else self._cdev(dU, torch.complex128),
                                 None if dUb is None else self._cdev(dUb, torch.complex128), self._stream())
        stats = res.solve.asdict()
        stats["tj"] = per_r.view(np.complex128).copy()  # per-RHS contractions of the forward solves
        out = (complex(res.tr[0], res.tr[1]), complex(g[0], g[1]), dU, dUb, stats)
        if st != OK and (check or st not in (ENOCONV, EBREAKDOWN)):
            self._err(st, out)
        return out

    def deflation(self, op, nvec, degree=0, max_outer=0, tol=0.0, seed=1, check=True):
        """Ritz vectors of the nvec smallest eigenvalues of A (Sec. Deflation).
        Returns a Deflation (with .evals, .resid, .outer, .subspace)."""
        eo = EigOpts()
        eo.degree, eo.max_outer, eo.tol, eo.seed = int(degree), int(max_outer), float(tol), int(seed)
        h = ctypes.c_void_p()
        st = lib().dp_deflation_create(self.h, ctypes.byref(op), int(nvec), ctypes.byref(eo), ctypes.byref(h),
                                       self._stream())
        d = Deflation(self, h, int(nvec), tuple(op.dims), int(op.nc)) if h.value else None
        if st != OK and (check or st != ENOCONV or d is None):
            if d is not None:
                d.close()
            self._err(st)
        return d

    def trace_deflated(self, op, defl, p, ps, opts, check=True):
        """Deflated probed estimate of Tr(P A^{-1}); dict as trace_estimate
        plus "T_defl" = Tr(P A^{-1} Q)."""
        res = TraceResult()
        ndil = ps.nc if ps.dilute else 1
        nrhs = ps.nsamples * ps.ncolors * ndil
        per_s, per_r = np.zeros(2 * ps.nsamples), np.zeros(2 * nrhs)
        res.per_sample = per_s.ctypes.data
        res.per_rhs = per_r.ctypes.data
        td = (ctypes.c_double * 2)()
        st = lib().dp_trace_deflated(self.h, ctypes.byref(op), defl.h, int(p), ctypes.byref(ps), ctypes.byref(opts),
                                     ctypes.byref(res), td, self._stream())
        out = {"T": complex(res.tr[0], res.tr[1]), "stderr": res.stderr_, "T_defl": complex(td[0], td[1]),
               "per_sample": per_s.view(np.complex128).copy(), "tj": per_r.view(np.complex128).copy(),
               "solve": res.solve.asdict()}
        if st != OK and (check or st not in (ENOCONV, EBREAKDOWN)):
            self._err(st, out)
        return out

    def solve_noalloc(self, op, b, opts, x=None, check=True):
        """One instance, b: complex128 [nrhs, N, nc]; the library allocates
        nothing (its workspace is a static device array)."""
        torch = self.torch
        if x is None:
            x = torch.empty_like(b)
        m = b.shape[0] * int(np.prod(list(op.dims))) * op.nc if min(op.dims) >= 1 else None
        stats = SolveStats()
        st = lib().dp_solve_noalloc(self.h, ctypes.byref(op), self._cdev(b, torch.complex128, m),
                                    self._cdev(x, torch.complex128, m), b.shape[0], ctypes.byref(opts),
                                    ctypes.byref(stats), self._stream())
        res = (x, stats.asdict())
        if st != OK and (check or st not in (ENOCONV, EBREAKDOWN)):
            self._err(st, res)
        return res

    def apply(self, op, v, prec="f64"):
        torch = self.torch
        y = torch.empty_like(v)
        m = v.shape[0] * int(np.prod(list(op.dims))) * op.nc
        st = lib().dp_apply(self.h, ctypes.byref(op), PREC[prec], self._cdev(v, torch.complex128, m),
                            self._cdev(y, torch.complex128, m), v.shape[0], self._stream())
        if st != OK:
            self._err(st)
        return y


class Deflation:
    """Deflation vectors of one operator, owned by the library (device memory)."""

    def __init__(self, ctx, h, nvec, dims, nc):
        self.ctx, self.h, self.nvec, self.dims, self.nc = ctx, h, nvec, tuple(int(v) for v in dims), nc
        ev, rs = np.zeros(nvec), np.zeros(nvec)
        outer, sub = ctypes.c_int32(), ctypes.c_int32()
        lib().dp_deflation_info(h, ev.ctypes.data, rs.ctypes.data, ctypes.byref(outer), ctypes.byref(sub))
        self.evals, self.resid, self.outer, self.subspace = ev, rs, int(outer.value), int(sub.value)

    def vectors(self, dims=None, nc=None):
        """The Ritz vectors, complex128 cuda tensor [nvec, N, nc] (dims and nc
        are those of the operator; if given they must match)."""
        torch = self.ctx.torch
        if (dims is not None and tuple(_dims4(dims)) != self.dims) or (nc is not None and nc != self.nc):
            raise ValueError(f"the deflation is for dims {self.dims}, nc {self.nc}")
        dims, nc = self.dims, self.nc
        N = int(np.prod(list(dims)))
        out = torch.empty((self.nvec, N, nc), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        st = lib().dp_deflation_vectors(self.ctx.h, self.h, self.ctx._cdev(out, torch.complex128),
                                        self.ctx._stream())
        if st != OK:
            self.ctx._err(st)
        return out

    def close(self):
        if self.h:
            lib().dp_deflation_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ctx_cache = {}


def context(device: int = 0) -> Context:
    if device not in _ctx_cache:
        _ctx_cache[device] = Context(device)
    return _ctx_cache[device]


def _make_probed_trace():
    import torch

    class ProbedTrace(torch.autograd.Function):
        """T = probed estimate of Tr(P A^{-1}) as a differentiable function of
        m2 (real scalar tensor) and the links U (complex128 [4, N, nc, nc]).

        Forward runs trace_estimate; backward recomputes the solves with
        trace_grad (no Krylov history is stored) and maps the Wirtinger pair
        (dT/dU, dT/dconj(U)) to PyTorch's convention for a complex output:
        grad_U = conj(g) dT/dconj(U) + g conj(dT/dU),
        grad_m2 = Re(conj(g) dT/dm2)."""

        @staticmethod
        def forward(ctx_, m2, U, dims, nc, p, colors_dev, ncolors, seed, sample0, nsamples, noise, dilute,
                    opts):
            c = context(U.device.index or 0)
            op = c.operator(dims, nc, float(m2), U.detach().contiguous())
            ps = c.probe_spec(dims, nc, colors_dev, ncolors, seed, sample0, nsamples, noise, dilute)
            r = c.trace_estimate([op], [ps], [p], opts)[0]
            ctx_.save_for_backward(m2, U)
            ctx_.args = (dims, nc, p, colors_dev, ncolors, seed, sample0, nsamples, noise, dilute, opts)
            return torch.tensor(r["T"], dtype=torch.complex128, device=U.device)

        @staticmethod
        def backward(ctx_, g):
            m2, U = ctx_.saved_tensors
            dims, nc, p, colors_dev, ncolors, seed, sample0, nsamples, noise, dilute, opts = ctx_.args
            c = context(U.device.index or 0)
            op = c.operator(dims, nc, float(m2), U.detach().contiguous())
            ps = c.probe_spec(dims, nc, colors_dev, ncolors, seed, sample0, nsamples, noise, dilute)
            _, dm2, dU, dUb, _ = c.trace_grad(op, ps, p, opts)
            gc = torch.conj(g)
            grad_U = gc * dUb + g * torch.conj(dU)
            grad_m2 = (gc * dm2).real.to(m2.dtype).reshape(m2.shape)
            return (grad_m2, grad_U) + (None,) * 11

    return ProbedTrace


def probed_trace(m2, U, dims, nc, p, colors_dev, ncolors, seed=0, sample0=0, nsamples=1, noise="z2_complex",
                 dilute=True, opts=None):
    """Differentiable probed estimate of Tr(P A^{-1}) (see ProbedTrace)."""
    if opts is None:
        opts = Context.opts(tol=1e-10)
    return _make_probed_trace().apply(m2, U, tuple(dims), nc, p, colors_dev, ncolors, seed, sample0, nsamples,
                                      noise, dilute, opts)
