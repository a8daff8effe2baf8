"""ctypes front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It loads oracle/libblp_oracle.so (plain C, FP64), which
shares no code with the HIP path.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class PrecOpts(C.Structure):
    _fields_ = [("corner", C.c_int), ("mg_fixed", C.c_int),
                ("mg_rtol", C.c_double), ("mg_maxcyc", C.c_int)]


class PrecStats(C.Structure):
    _fields_ = [("applies", C.c_long), ("mg_cycles_total", C.c_long),
                ("mg_cycles_min", C.c_int), ("mg_cycles_max", C.c_int)]


class GmresOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("absolute", C.c_int), ("restart", C.c_int),
                ("maxit", C.c_int), ("precond", C.c_int), ("transpose", C.c_int),
                ("scaled", C.c_int), ("prec", PrecOpts), ("stop_on_estimate", C.c_int)]


class GmresInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("true_res", C.c_double), ("norm_F", C.c_double),
                ("mg_cycles_total", C.c_long), ("mg_cycles_min", C.c_int),
                ("mg_cycles_max", C.c_int)]


class Gmres1Opts(C.Structure):
    _fields_ = [("K", C.c_double), ("g", C.c_double), ("maxit", C.c_int), ("left", C.c_int)]


class Gmres1Info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("res_inf", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        path = _build.build_oracle(force=False)
        L = C.CDLL(path)
        L.orc_mesh_axis.restype = C.c_double
        L.orc_mesh_axis.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                 _dp, _dp, _dp]
        L.orc_mesh_axis_ex.restype = C.c_double
        L.orc_mesh_axis_ex.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int,
                                       C.c_int, _dp, _dp]
        L.orc_create_ex.restype = C.c_void_p
        L.orc_create_ex.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_mesh_axis_layer.restype = C.c_double
        L.orc_mesh_axis_layer.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int,
                                          C.c_int, C.c_int, _dp, _dp]
        L.orc_create_px.restype = C.c_void_p
        L.orc_create_px.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        for f in ("orc_y_layer", "orc_par_num_levels"):
            getattr(L, f).restype = C.c_int
            getattr(L, f).argtypes = [C.c_void_p]
        L.orc_par_level_nx.restype = C.c_int
        L.orc_par_level_nx.argtypes = [C.c_void_p, C.c_int]
        L.orc_par_level_stencil.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_par_level_weights.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        for f in ("orc_par_level_apply", "orc_par_level_gs", "orc_par_level_restrict",
                  "orc_par_level_interp"):
            getattr(L, f).argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_par_corner_mg.restype = C.c_int
        L.orc_par_corner_mg.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, _dp, _dp]
        for f in ("orc_n", "orc_num_levels"):
            getattr(L, f).restype = C.c_int
            getattr(L, f).argtypes = [C.c_void_p]
        L.orc_level_size.restype = C.c_int
        L.orc_level_size.argtypes = [C.c_void_p, C.c_int]
        L.orc_nodes.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_stencil.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp]
        L.orc_apply_A.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_apply_AT.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_csr.restype = C.c_int
        L.orc_csr.argtypes = [C.c_void_p, _ip, _ip, _dp]
        L.orc_prec_apply.argtypes = [C.c_void_p, C.POINTER(PrecOpts), C.c_int, _dp, _dp,
                                     C.POINTER(PrecStats)]
        for f in ("orc_solve_I", "orc_solve_Y", "orc_solve_X"):
            getattr(L, f).argtypes = [C.c_void_p, _dp, _dp]
        L.orc_corner_mg.restype = C.c_int
        L.orc_corner_mg.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int,
                                    _dp, _dp]
        L.orc_corner_exact.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        for f in ("orc_level_apply", "orc_level_restrict", "orc_level_interp",
                  "orc_level_gs"):
            getattr(L, f).argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_fgmres.restype = C.c_int
        L.orc_fgmres.argtypes = [C.c_void_p, C.POINTER(GmresOpts), _dp, _dp,
                                 C.POINTER(GmresInfo), _dp]
        L.orc_sine_series.argtypes = [C.c_int, _dp, _dp, C.c_int, C.c_int, _dp, _dp]
        L.orc_sine_project.argtypes = [C.c_int, _dp, _dp, C.c_int, C.c_int, _dp, _dp]
        L.orc_bilinear.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp, _dp]
        L.orc_bilinear_project.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp, _dp]
        L.orc1_create.restype = C.c_void_p
        L.orc1_create.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp, C.c_int]
        L.orc1_destroy.argtypes = [C.c_void_p]
        L.orc1_n.restype = C.c_int
        L.orc1_n.argtypes = [C.c_void_p]
        L.orc1_stencil.argtypes = [C.c_void_p, C.c_int, _dp]
        for f in ("orc1_apply_A", "orc1_solve_A", "orc1_prec_apply"):
            getattr(L, f).argtypes = [C.c_void_p, _dp, _dp]
        L.orc1_prec_matrix.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc1_gmres.restype = C.c_int
        L.orc1_gmres.argtypes = [C.c_void_p, C.POINTER(Gmres1Opts), _dp, _dp,
                                 C.POINTER(Gmres1Info), _dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


MESH_KINDS = {"shishkin": 0, "bakhvalov-shishkin": 1}
LAYERS = {"exponential": 0, "parabolic": 1}


def mesh_axis(N, eps, sigma=2.0, clow=1.0, kind="shishkin", layer_cells=None,
              layer="exponential"):
    """One axis of the layer-adapted mesh: (tau, nodes[0..N], widths[0..N]).
    kind 'shishkin' or 'bakhvalov-shishkin'; layer_cells = cells on [0, tau]
    (default N/2); layer 'exponential' (width scale eps/clow) or 'parabolic'
    (sqrt(eps))."""
    nodes = np.zeros(N + 1)
    widths = np.zeros(N + 2)
    nl = N // 2 if layer_cells is None else int(layer_cells)
    tau = lib().orc_mesh_axis_layer(N, eps, sigma, clow, MESH_KINDS[kind], nl, LAYERS[layer],
                                    _p(nodes), _p(widths))
    return tau, nodes, widths[: N + 1]


class Problem:
    """Upwind 5-point operator on the tensor Shishkin mesh, plus the
    boundary-layer preconditioner and FGMRES of the paper (FP64, CPU)."""

    def __init__(self, N, eps, c1=None, c2=None, r=None, sigma=2.0, clow_x=1.0,
                 clow_y=1.0, mesh_kind="shishkin", layer_cells=None, y_layer="exponential"):
        self.N, self.eps, self.n1 = N, eps, N - 1
        nl = N // 2 if layer_cells is None else int(layer_cells)
        self.y_layer = y_layer
        tx, self.x, self.hx = mesh_axis(N, eps, sigma, clow_x, mesh_kind, nl)
        ty, self.y, self.hy = mesh_axis(N, eps, sigma, clow_y, mesh_kind, nl, layer=y_layer)
        self.tau_x, self.tau_y = tx, ty
        c1x = _f64(c1(self.x) if callable(c1) else (np.ones(N + 1) if c1 is None else c1))
        c2y = _f64(c2(self.y) if callable(c2) else (np.ones(N + 1) if c2 is None else c2))
        if r is None:
            rr = np.ones(self.n1 * self.n1)
        elif np.isscalar(r):
            rr = np.full(self.n1 * self.n1, float(r))
        else:
            rr = _f64(r).ravel()
        self.c1x, self.c2y, self.r = c1x, c2y, rr
        self._h = lib().orc_create_px(N, eps, sigma, clow_x, clow_y, MESH_KINDS[mesh_kind], nl,
                                      LAYERS[y_layer], _p(c1x), _p(c2y), _p(rr))
        if not self._h:
            raise ValueError("orc_create_px rejected N=%r, layer cells %r" % (N, nl))
        self.n = self.n1 * self.n1
        self.h = nl

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and _lib is not None:  # (at interpreter exit the library may be gone)
            _lib.orc_destroy(h)

    @property
    def levels(self):
        return [lib().orc_level_size(self._h, l) for l in range(lib().orc_num_levels(self._h))]

    def stencil(self, i, j):
        out = np.zeros(5)
        lib().orc_stencil(self._h, i, j, _p(out))
        return dict(zip(("W", "E", "S", "N", "C"), out))

    def A(self, x):
        x = _f64(x)
        y = np.zeros(self.n)
        lib().orc_apply_A(self._h, _p(x), _p(y))
        return y

    def AT(self, x):
        x = _f64(x)
        y = np.zeros(self.n)
        lib().orc_apply_AT(self._h, _p(x), _p(y))
        return y

    def csr(self):
        import scipy.sparse as sp
        rowptr = np.zeros(self.n + 1, dtype=np.int32)
        col = np.zeros(5 * self.n, dtype=np.int32)
        val = np.zeros(5 * self.n)
        nnz = lib().orc_csr(self._h, rowptr.ctypes.data_as(_ip), col.ctypes.data_as(_ip), _p(val))
        return sp.csr_matrix((val[:nnz], col[:nnz], rowptr), shape=(self.n, self.n))

    @staticmethod
    def prec_opts(corner="mg", mg_fixed=0, mg_rtol=1e-3, mg_maxcyc=20):
        return PrecOpts(0 if corner == "exact" else 1, mg_fixed, mg_rtol, mg_maxcyc)

    def M_inv(self, b, transpose=False, **kw):
        b = _f64(b)
        z = np.zeros(self.n)
        st = PrecStats()
        o = self.prec_opts(**kw)
        lib().orc_prec_apply(self._h, C.byref(o), int(transpose), _p(b), _p(z), C.byref(st))
        self.last_prec_stats = st
        return z

    def solve_region(self, name, b, z):
        b = _f64(b)
        z = _f64(z).copy()
        getattr(lib(), "orc_solve_" + name)(self._h, _p(b), _p(z))
        return z

    def corner_mg(self, bC, transpose=False, fixed=0, rtol=1e-3, maxcyc=20):
        """The corner multigrid of the problem's layer type (the parabolic one
        has no transposed form)."""
        bC = _f64(bC)
        z = np.zeros_like(bC)
        if self.y_layer == "parabolic":
            if transpose:
                raise ValueError("the parabolic corner cycle has no transposed form")
            cyc = lib().orc_par_corner_mg(self._h, fixed, rtol, maxcyc, _p(bC), _p(z))
        else:
            cyc = lib().orc_corner_mg(self._h, int(transpose), fixed, rtol, maxcyc, _p(bC),
                                      _p(z))
        return z, cyc

    # parabolic-case semicoarsening hierarchy (level l: nx_l x h nodes) -----
    @property
    def par_levels(self):
        return [lib().orc_par_level_nx(self._h, l) for l in range(lib().orc_par_num_levels(self._h))]

    def par_stencil(self, l):
        """9-point stencils of level l, array [j-1, i-1, dj+1, di+1]."""
        nx = self.par_levels[l]
        a = np.zeros(9 * nx * self.h)
        lib().orc_par_level_stencil(self._h, l, _p(a))
        return a.reshape(self.h, nx, 3, 3)

    def par_weights(self, l):
        nx = self.par_levels[l]
        wl, wr = np.zeros(nx * self.h), np.zeros(nx * self.h)
        lib().orc_par_level_weights(self._h, l, _p(wl), _p(wr))
        return wl.reshape(self.h, nx), wr.reshape(self.h, nx)

    def par_op(self, name, l, v, z=None):
        sizes = self.par_levels
        v = _f64(v)
        if name == "gs":
            out = _f64(z).copy()
        elif name == "restrict":
            out = np.zeros(sizes[l + 1] * self.h)
        else:
            out = np.zeros(sizes[l] * self.h)
        getattr(lib(), "orc_par_level_" + name)(self._h, l, _p(v), _p(out))
        return out

    def corner_exact(self, bC, transpose=False):
        bC = _f64(bC)
        z = np.zeros_like(bC)
        lib().orc_corner_exact(self._h, int(transpose), _p(bC), _p(z))
        return z

    def level_op(self, name, l, v):
        sizes = self.levels
        v = _f64(v)
        if name == "restrict":
            out = np.zeros(sizes[l + 1] ** 2)
        else:
            out = np.zeros(sizes[l] ** 2)
        getattr(lib(), "orc_level_" + name)(self._h, l, _p(v), _p(out))
        return out

    def level_gs(self, l, b, z):
        b = _f64(b)
        z = _f64(z).copy()
        lib().orc_level_gs(self._h, l, _p(b), _p(z))
        return z

    def fgmres(self, F, tol=1e-8, restart=50, maxit=1000, precond=True, transpose=False,
               absolute=False, scaled=False, corner="mg", mg_fixed=0, mg_rtol=1e-3,
               mg_maxcyc=20, stop_on_estimate=False):
        F = _f64(F)
        u = np.zeros(self.n)
        o = GmresOpts(tol, int(absolute), restart, maxit, int(precond), int(transpose),
                      int(scaled), self.prec_opts(corner, mg_fixed, mg_rtol, mg_maxcyc),
                      int(stop_on_estimate))
        info = GmresInfo()
        hist = np.zeros(maxit + 1)
        status = lib().orc_fgmres(self._h, C.byref(o), _p(F), _p(u), C.byref(info), _p(hist))
        return u, status, info, hist[: info.iterations + 1]

    # grid helpers ---------------------------------------------------------
    def grid(self, v):
        """(N-1)^2 vector -> array indexed [j-1, i-1]."""
        return np.asarray(v).reshape(self.n1, self.n1)


def sine_series(N, x, y, a):
    a = _f64(a)
    L, K = a.shape  # a[l-1, k-1]
    F = np.zeros((N - 1) ** 2)
    lib().orc_sine_series(N, _p(_f64(x)), _p(_f64(y)), K, L, _p(a), _p(F))
    return F


def sine_project(N, x, y, lam, K, L):
    g = np.zeros(K * L)
    lib().orc_sine_project(N, _p(_f64(x)), _p(_f64(y)), K, L, _p(_f64(lam)), _p(g))
    return g.reshape(L, K)


def bilinear(N, x, y, R):
    R = _f64(R)
    m = R.shape[0]
    r = np.zeros((N - 1) ** 2)
    lib().orc_bilinear(N, _p(_f64(x)), _p(_f64(y)), m, _p(R), _p(r))
    return r


def bilinear_project(N, x, y, w, m):
    G = np.zeros(m * m)
    lib().orc_bilinear_project(N, _p(_f64(x)), _p(_f64(y)), m, _p(_f64(w)), _p(G))
    return G.reshape(m, m)


class Problem1D:
    """The one-dimensional method of Sec. 2 (FP64, CPU): upwind stencil on a
    layer-adapted mesh, the block preconditioner M of eq. block_M and
    unrestarted GMRES with the inf-norm residual test of Sec. 2.4.  c and r
    are callables of x or arrays of the N+1 nodal values."""

    def __init__(self, N, eps, c, r, sigma=2.0, clow=1.0, mesh_kind="shishkin",
                 layer_cells=None):
        self.N, self.eps, self.n = N, eps, N - 1
        self.nl = N // 2 if layer_cells is None else int(layer_cells)
        self.tau, self.x, w = mesh_axis(N, eps, sigma, clow, mesh_kind, self.nl)
        self.w = np.zeros(N + 2)
        self.w[: N + 1] = w
        cv = _f64(c(self.x) if callable(c) else c)
        rv = _f64(r(self.x) if callable(r) else (np.full(N + 1, float(r)) if np.isscalar(r) else r))
        self.c, self.r = cv, rv
        self._h = lib().orc1_create(N, eps, _p(self.w), _p(cv), _p(rv), self.nl)
        if not self._h:
            raise ValueError("orc1_create rejected N=%r, layer cells %r" % (N, self.nl))

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and _lib is not None:
            _lib.orc1_destroy(h)

    def stencil(self, i):
        out = np.zeros(3)
        lib().orc1_stencil(self._h, i, _p(out))
        return out

    def _op(self, name, v):
        v = _f64(v)
        y = np.zeros(self.n)
        getattr(lib(), name)(self._h, _p(v), _p(y))
        return y

    def A(self, v):
        return self._op("orc1_apply_A", v)

    def solve(self, f):
        return self._op("orc1_solve_A", f)

    def M_inv(self, b):
        return self._op("orc1_prec_apply", b)

    def M_tridiag(self):
        a, d, e = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        lib().orc1_prec_matrix(self._h, _p(a), _p(d), _p(e))
        return a, d, e

    def dense(self):
        A = np.zeros((self.n, self.n))
        for k in range(self.n):
            W, Cc, E = self.stencil(k + 1)
            A[k, k] = Cc
            if k > 0:
                A[k, k - 1] = W
            if k < self.n - 1:
                A[k, k + 1] = E
        return A

    def gmres(self, F, K, g, maxit=200, left=True):
        F = _f64(F)
        u = np.zeros(self.n)
        info = Gmres1Info()
        hist = np.zeros(maxit + 1)
        st = lib().orc1_gmres(self._h, C.byref(Gmres1Opts(K, g, maxit, int(left))), _p(F), _p(u),
                              C.byref(info), _p(hist))
        return u, st, info, hist[: info.iterations + 1]
