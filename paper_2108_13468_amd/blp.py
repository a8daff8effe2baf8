"""Python binding of the HIP library libblp.so (C ABI in include/blp.h).

Argument marshalling only: device buffers are torch tensors on the HIP
device (their data_ptr() is passed), host arrays are numpy arrays, and the
problem's stream is torch's current stream at assemble time.  Every step of
the solver runs in the library's kernels.  There is no fallback: if the
library is not built, loading raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libblp.so")

BLP_OK, BLP_W_NOCONV = 0, 1
BLP_CONST, BLP_AXIS, BLP_NODAL, BLP_BILINEAR = 0, 1, 2, 3
BLP_FP64, BLP_MIXED = 0, 1
OPS = {"A": 0, "AT": 1, "MINV": 2, "MINVT": 3, "MINV32": 4}

# Symbols declared in include/blp.h (checked by the CPU tests).
EXPORTS = ("blp_mesh", "blp_assemble", "blp_nodes", "blp_precondition", "blp_solve",
           "blp_solve_adjoint", "blp_apply", "blp_sine_rhs", "blp_sine_project",
           "blp_bilinear_project", "blp_mul", "blp_reaction_gradient", "blp_sine_project_noalloc",
           "blp1d_solve", "blp_timing", "blp_footprint", "blp_destroy",
           "blp_strerror", "blp_batch_create", "blp_batch_solve", "blp_batch_solve_adjoint",
           "blp_batch_footprint", "blp_batch_describe", "blp_batch_timing", "blp_batch_destroy")
NCLASS = 7
CLASSES = ("sweep", "gs_rhs", "lines", "mg_other", "spmv", "krylov", "layout")

_dp = C.POINTER(C.c_double)


class Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("m", C.c_int), ("v", _dp)]


class MeshOpts(C.Structure):
    _fields_ = [("sigma", C.c_double), ("clow_x", C.c_double), ("clow_y", C.c_double),
                ("kind", C.c_int), ("layer_cells", C.c_int), ("y_layer", C.c_int)]


MESH_KINDS = {"shishkin": 0, "bakhvalov-shishkin": 1}
Y_LAYERS = {"exponential": 0, "parabolic": 1}


def _mesh_opts(sigma, clow, kind, layer_cells, y_layer="exponential"):
    return MeshOpts(sigma, clow[0], clow[1], MESH_KINDS[kind], int(layer_cells or 0),
                    Y_LAYERS[y_layer])


class PrecOpts(C.Structure):
    _fields_ = [("mg_fixed", C.c_int), ("mg_rtol", C.c_double), ("mg_maxcyc", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("absolute", C.c_int), ("scaled", C.c_int),
                ("restart", C.c_int), ("maxit", C.c_int), ("precision", C.c_int),
                ("precond", C.c_int), ("stop_on_estimate", C.c_int)]


class BatchOpts(C.Structure):
    _fields_ = [("graphs", C.c_int), ("autotune", C.c_int), ("sweep_variant", C.c_int)]


class Problem1D(C.Structure):
    # c and r: addresses of host double arrays (const double * in the C ABI)
    _fields_ = [("N", C.c_int), ("eps", C.c_double), ("sigma", C.c_double), ("clow", C.c_double),
                ("kind", C.c_int), ("layer_cells", C.c_int), ("c", C.c_void_p), ("r", C.c_void_p)]


class Opts1D(C.Structure):
    _fields_ = [("maxit", C.c_int), ("left", C.c_int), ("K", C.c_double), ("g", C.c_double)]


class Info1D(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("res_inf", C.c_double),
                ("K", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("res", C.c_double), ("norm_F", C.c_double), ("mg_cycles_total", C.c_long),
                ("mg_cycles_min", C.c_int), ("mg_cycles_max", C.c_int),
                ("solve_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BlpError(RuntimeError):
    """A negative status of the library; .code holds it."""

    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


_lib = None


def lib():
    """Load libblp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch first: its HIP runtime and the one libblp.so links against share
        # the soname libamdhip64.so.7, so loading torch first makes the dynamic
        # loader bind libblp.so to the same runtime instance (one device context
        # per process instead of two).
        import torch  # noqa: F401
        if not os.path.exists(LIBPATH):
            raise BlpError("libblp.so not built: run __graft_entry__.build() "
                           "(or python paper_2108_13468_amd/build.py)")
        L = C.CDLL(LIBPATH)
        vp = C.c_void_p
        L.blp_mesh.argtypes = [C.c_int, C.c_double, C.POINTER(MeshOpts), _dp, _dp, _dp]
        L.blp_assemble.argtypes = [C.c_int, C.c_double, C.POINTER(Field), C.POINTER(Field),
                                   C.POINTER(Field), C.POINTER(MeshOpts), vp, C.POINTER(vp)]
        L.blp_nodes.argtypes = [vp, _dp, _dp]
        L.blp_precondition.argtypes = [vp, C.POINTER(PrecOpts)]
        for f in ("blp_solve", "blp_solve_adjoint"):
            getattr(L, f).argtypes = [vp, C.c_int, vp, vp, C.POINTER(SolveOpts),
                                      C.POINTER(SolveInfo), _dp]
        L.blp_apply.argtypes = [vp, C.c_int, vp, vp, C.POINTER(C.c_int)]
        L.blp_sine_rhs.argtypes = [vp, C.c_int, C.c_int, _dp, vp]
        L.blp_sine_project.argtypes = [vp, C.c_int, C.c_int, vp, _dp]
        L.blp_sine_project_noalloc.argtypes = [vp, C.c_int, C.c_int, vp, _dp]
        L.blp_bilinear_project.argtypes = [vp, C.c_int, vp, _dp]
        L.blp_mul.argtypes = [vp, vp, vp, vp]
        L.blp_reaction_gradient.argtypes = [vp, C.c_int, C.c_int, vp, vp, _dp]
        L.blp_timing.argtypes = [vp, C.c_int, _dp, C.POINTER(C.c_longlong), _dp]
        L.blp_footprint.restype = C.c_longlong
        L.blp_footprint.argtypes = [vp]
        L.blp_destroy.argtypes = [vp]
        L.blp_strerror.restype = C.c_char_p
        L.blp_strerror.argtypes = [C.c_int]
        L.blp_batch_create.argtypes = [C.POINTER(vp), C.c_int, vp, C.POINTER(BatchOpts),
                                       C.POINTER(vp)]
        for f in ("blp_batch_solve", "blp_batch_solve_adjoint"):
            getattr(L, f).argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(SolveOpts),
                                      C.POINTER(SolveInfo)]
        L.blp_batch_describe.argtypes = [vp, C.c_char_p, C.c_int]
        L.blp_batch_timing.argtypes = [vp, C.c_int, _dp, C.POINTER(C.c_longlong), _dp]
        L.blp_batch_footprint.restype = C.c_longlong
        L.blp_batch_footprint.argtypes = [vp]
        L.blp_batch_destroy.argtypes = [vp]
        L.blp1d_solve.argtypes = [C.c_int, C.POINTER(Problem1D), C.POINTER(vp), C.POINTER(vp),
                                  C.POINTER(Opts1D), vp, C.POINTER(Info1D)]
        _lib = L
    return _lib


def _check(rc, what):
    if rc < 0:
        raise BlpError("%s failed: %s (%d)" % (what, lib().blp_strerror(rc).decode(), rc), rc)
    return rc


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def mesh(N, eps, sigma=2.0, clow=(1.0, 1.0), kind="shishkin", layer_cells=None,
         y_layer="exponential"):
    """Mesh nodes of both axes: ((tau_x, tau_y), x[0..N], y[0..N]); y_layer
    'parabolic' takes the transition point sigma sqrt(eps) ln N on y."""
    x, y, tau = np.zeros(N + 1), np.zeros(N + 1), np.zeros(2)
    o = _mesh_opts(sigma, clow, kind, layer_cells, y_layer)
    _check(lib().blp_mesh(N, eps, C.byref(o), x.ctypes.data_as(_dp), y.ctypes.data_as(_dp),
                          tau.ctypes.data_as(_dp)), "blp_mesh")
    return (float(tau[0]), float(tau[1])), x, y


def _field(spec, N, keep):
    """spec: float (constant), ('axis', values[N+1]), ('nodal', values[(N-1)^2]),
    ('bilinear', controls[m, m] indexed [q, p])."""
    if np.isscalar(spec):
        arr, kind, m = _f64([spec]), BLP_CONST, 0
    else:
        tag, vals = spec
        arr = _f64(vals).ravel()
        kind = {"axis": BLP_AXIS, "nodal": BLP_NODAL, "bilinear": BLP_BILINEAR}[tag]
        m = int(np.asarray(vals).shape[0]) if tag == "bilinear" else 0
    keep.append(arr)
    return Field(kind, m, arr.ctypes.data_as(_dp))


class Problem:
    """An assembled operator on the device (one handle of the C library)."""

    def __init__(self, N, eps, c1, c2, r, sigma=2.0, clow=(1.0, 1.0), stream=None,
                 mesh_kind="shishkin", layer_cells=None, y_layer="exponential"):
        import torch
        self.torch = torch
        self.N, self.eps, self.n = N, eps, (N - 1) ** 2
        self.device = torch.device("cuda", torch.cuda.current_device())
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        keep = []
        f1, f2, fr = _field(c1, N, keep), _field(c2, N, keep), _field(r, N, keep)
        mo = _mesh_opts(sigma, clow, mesh_kind, layer_cells, y_layer)
        self.y_layer = y_layer
        h = C.c_void_p()
        _check(lib().blp_assemble(N, eps, C.byref(f1), C.byref(f2), C.byref(fr), C.byref(mo),
                                  C.c_void_p(stream.cuda_stream), C.byref(h)), "blp_assemble")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and _lib is not None:  # (at interpreter exit the library may be gone)
            _lib.blp_destroy(h)

    __del__ = close

    def nodes(self):
        x, y = np.zeros(self.N + 1), np.zeros(self.N + 1)
        _check(lib().blp_nodes(self._h, x.ctypes.data_as(_dp), y.ctypes.data_as(_dp)), "blp_nodes")
        return x, y

    def precondition(self, mg_fixed=0, mg_rtol=None, mg_maxcyc=20):
        """mg_rtol None: the paper's corner reduction, 1e-3 for two
        exponential layers, 1e-2 with a parabolic layer (Sec. 3.2)."""
        if mg_rtol is None:
            mg_rtol = 1e-2 if self.y_layer == "parabolic" else 1e-3
        o = PrecOpts(mg_fixed, mg_rtol, mg_maxcyc)
        _check(lib().blp_precondition(self._h, C.byref(o)), "blp_precondition")
        return self

    def _vec(self, x, nrhs=None):
        t = self.torch
        if not (isinstance(x, t.Tensor) and x.is_cuda and x.dtype == t.float64 and x.is_contiguous()):
            raise TypeError("expected a contiguous float64 tensor on the HIP device")
        if x.numel() % self.n:
            raise ValueError("vector length must be a multiple of (N-1)^2")
        return x

    def _solve(self, fn, F, tol, scaled, restart, maxit, precision, precond, absolute, hist,
               stop_on_estimate=False):
        t = self.torch
        F = self._vec(F)
        nrhs = F.numel() // self.n
        U = t.empty_like(F)
        o = SolveOpts(tol, int(absolute), int(scaled), restart, maxit,
                      BLP_MIXED if precision == "mixed" else BLP_FP64, int(precond),
                      int(stop_on_estimate))
        infos = (SolveInfo * nrhs)()
        h = np.zeros(nrhs * (maxit + 1)) if hist else None
        rc = _check(fn(self._h, nrhs, C.c_void_p(F.data_ptr()), C.c_void_p(U.data_ptr()),
                       C.byref(o), infos, h.ctypes.data_as(_dp) if hist else None), "solve")
        out = [i.as_dict() for i in infos]
        for d in out:
            d["status"] = rc
        if hist:
            return U, out, h.reshape(nrhs, maxit + 1)
        return U, out

    def solve(self, F, tol=1e-8, scaled=True, restart=50, maxit=1000, precision="fp64",
              precond=True, absolute=False, hist=False, stop_on_estimate=False):
        return self._solve(lib().blp_solve, F, tol, scaled, restart, maxit, precision, precond,
                           absolute, hist, stop_on_estimate)

    def solve_adjoint(self, G, tol=1e-8, scaled=True, restart=50, maxit=1000, precision="fp64",
                      precond=True, absolute=False, hist=False, stop_on_estimate=False):
        return self._solve(lib().blp_solve_adjoint, G, tol, scaled, restart, maxit, precision,
                           precond, absolute, hist, stop_on_estimate)

    def apply(self, op, x):
        x = self._vec(x)
        y = self.torch.empty_like(x)
        cyc = C.c_int(0)
        _check(lib().blp_apply(self._h, OPS[op], C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                               C.byref(cyc)), "blp_apply")
        self.last_cycles = cyc.value
        return y

    def sine_rhs(self, a, out=None):
        """F from sine coefficients a (L x K); with out, written into that
        contiguous float64 device vector of length (N-1)^2."""
        a = _f64(a)
        L, K = a.shape
        F = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device) if out is None \
            else out
        if F.numel() != self.n:
            raise ValueError("out must hold (N-1)^2 values")
        _check(lib().blp_sine_rhs(self._h, K, L, a.ctypes.data_as(_dp),
                                  C.c_void_p(self._vec(F).data_ptr())), "blp_sine_rhs")
        return F

    def sine_project(self, w, K, L):
        g = np.zeros(K * L)
        _check(lib().blp_sine_project(self._h, K, L, C.c_void_p(self._vec(w).data_ptr()),
                                      g.ctypes.data_as(_dp)), "blp_sine_project")
        return g.reshape(L, K)

    def sine_project_noalloc(self, w, K, L):
        """As sine_project, through the allocation-free entry point (fixed
        scratch array; raises BlpError with code -6 when it does not fit)."""
        g = np.zeros(K * L)
        _check(lib().blp_sine_project_noalloc(self._h, K, L, C.c_void_p(self._vec(w).data_ptr()),
                                              g.ctypes.data_as(_dp)), "blp_sine_project_noalloc")
        return g.reshape(L, K)

    def bilinear_project(self, w, m):
        G = np.zeros(m * m)
        _check(lib().blp_bilinear_project(self._h, m, C.c_void_p(self._vec(w).data_ptr()),
                                          G.ctypes.data_as(_dp)), "blp_bilinear_project")
        return G.reshape(m, m)

    def reaction_gradient(self, lam, U, m):
        """dJ/dR (m x m) from the adjoint solutions lam and solutions U
        (nrhs stacked vectors each): -sum over right-hand sides and nodes of
        lam u phi_p(x) phi_q(y)."""
        lam, U = self._vec(lam.reshape(-1)), self._vec(U.reshape(-1))
        if lam.numel() != U.numel():
            raise ValueError("lam and U must hold the same number of vectors")
        G = np.zeros(m * m)
        _check(lib().blp_reaction_gradient(self._h, m, lam.numel() // self.n,
                                           C.c_void_p(lam.data_ptr()), C.c_void_p(U.data_ptr()),
                                           G.ctypes.data_as(_dp)), "blp_reaction_gradient")
        return G.reshape(m, m)

    def mul(self, a, b):
        out = self.torch.empty_like(a)
        _check(lib().blp_mul(self._h, C.c_void_p(self._vec(a).data_ptr()),
                             C.c_void_p(self._vec(b).data_ptr()), C.c_void_p(out.data_ptr())),
               "blp_mul")
        return out

    def timing(self, enable):
        """enable=True starts per-kernel-class event timing; enable=False stops
        it and returns {class: (ms, launches, algorithmic bytes)}."""
        ms = np.zeros(NCLASS)
        nl = (C.c_longlong * NCLASS)()
        by = np.zeros(NCLASS)
        _check(lib().blp_timing(self._h, int(bool(enable)), ms.ctypes.data_as(_dp), nl,
                                by.ctypes.data_as(_dp)), "blp_timing")
        if enable:
            return None
        return {c: (float(ms[k]), int(nl[k]), float(by[k])) for k, c in enumerate(CLASSES)}

    def footprint(self):
        return int(lib().blp_footprint(self._h))


def from_instance(inst, nodal_r=None):
    """Assemble a problem from an inputs.Instance (coefficients sampled at the
    mesh nodes, which blp_mesh returns)."""
    _, x, y = mesh(inst.N, inst.eps, inst.sigma, inst.clow, inst.mesh_kind, inst.layer_cells,
                   inst.y_layer)
    if inst.r_ctrl is not None:
        r = ("bilinear", inst.r_ctrl)
    elif nodal_r is not None:
        r = ("nodal", nodal_r)
    else:
        r = float(inst.r_const)
    return Problem(inst.N, inst.eps, ("axis", inst.c1_at(x)), ("axis", inst.c2_at(y)), r,
                   sigma=inst.sigma, clow=inst.clow, mesh_kind=inst.mesh_kind,
                   layer_cells=inst.layer_cells, y_layer=inst.y_layer)


class Batch:
    """Independent systems solved together (blp_batch_*): one system per
    entry of `problems` (preconditioned Problems; a Problem may appear
    several times, once per right-hand side).  Runs on torch's current
    stream at creation."""

    def __init__(self, problems, graphs=False, autotune=False, sweep_variant=0):
        import torch
        self.torch = torch
        self.problems = list(problems)  # kept alive while the batch exists
        S = len(self.problems)
        arr = (C.c_void_p * S)(*[p._h for p in self.problems])
        stream = torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().blp_batch_create(arr, S, C.c_void_p(stream.cuda_stream),
                                      C.byref(BatchOpts(int(graphs), int(autotune),
                                                        int(sweep_variant))), C.byref(h)),
               "blp_batch_create")
        self._h = h
        self.S = S

    def close(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and _lib is not None:
            _lib.blp_batch_destroy(h)

    __del__ = close

    def _solve(self, fn, F, U, tol, scaled, restart, maxit, precision, precond, absolute):
        if len(F) != self.S:
            raise ValueError("one right-hand side per system")
        F = [p._vec(f) for p, f in zip(self.problems, F)]
        U = [self.torch.empty_like(f) for f in F] if U is None else [p._vec(u) for p, u in
                                                                        zip(self.problems, U)]
        o = SolveOpts(tol, int(absolute), int(scaled), restart, maxit,
                      BLP_MIXED if precision == "mixed" else BLP_FP64, int(precond), 0)
        infos = (SolveInfo * self.S)()
        fa = (C.c_void_p * self.S)(*[f.data_ptr() for f in F])
        ua = (C.c_void_p * self.S)(*[u.data_ptr() for u in U])
        rc = _check(fn(self._h, fa, ua, C.byref(o), infos), "batch solve")
        out = [i.as_dict() for i in infos]
        for d in out:
            d["status"] = rc
        return U, out

    def solve(self, F, U=None, tol=1e-8, scaled=True, restart=50, maxit=1000, precision="fp64",
              precond=True, absolute=False):
        return self._solve(lib().blp_batch_solve, F, U, tol, scaled, restart, maxit, precision,
                           precond, absolute)

    def solve_adjoint(self, G, L=None, tol=1e-8, scaled=True, restart=50, maxit=1000,
                      precision="fp64", precond=True, absolute=False):
        return self._solve(lib().blp_batch_solve_adjoint, G, L, tol, scaled, restart, maxit,
                           precision, precond, absolute)

    def footprint(self):
        return int(lib().blp_batch_footprint(self._h))

    def timing(self, enable):
        """As Problem.timing, for the batch's launches."""
        ms = np.zeros(NCLASS)
        nl = (C.c_longlong * NCLASS)()
        by = np.zeros(NCLASS)
        _check(lib().blp_batch_timing(self._h, int(bool(enable)), ms.ctypes.data_as(_dp), nl,
                                      by.ctypes.data_as(_dp)), "blp_batch_timing")
        if enable:
            return None
        return {c: (float(ms[k]), int(nl[k]), float(by[k])) for k, c in enumerate(CLASSES)}

    def describe(self):
        """Mesh classes and the kernel variants of the launch plans."""
        buf = C.create_string_buffer(8192)
        _check(lib().blp_batch_describe(self._h, buf, len(buf)), "blp_batch_describe")
        return buf.value.decode()


def solve_1d(problems, F, maxit=100, left=True, K=0.0, g=0.0, U=None):
    """The 1D method (Sec. 2) for a batch in one launch (blp1d_solve).
    problems: list of dicts with N, eps, c, r (arrays of N+1 nodal values)
    and optionally sigma (2), clow (1), kind ('shishkin'), layer_cells (N/2);
    F: list of float64 device tensors of N-1 values.  Returns (U, infos)."""
    import torch
    S = len(problems)
    if len(F) != S:
        raise ValueError("one right-hand side per problem")
    # the problem records as one numpy array laid out as blp1d_problem
    # (filled column by column); the c and r arrays stay referenced by keep
    keep = [(_f64(q["c"]), _f64(q["r"])) for q in problems]
    rec = np.zeros(S, dtype=np.dtype(Problem1D))
    rec["N"] = [q["N"] for q in problems]
    rec["eps"] = [q["eps"] for q in problems]
    rec["sigma"] = [q.get("sigma", 2.0) for q in problems]
    rec["clow"] = [q.get("clow", 1.0) for q in problems]
    rec["kind"] = [MESH_KINDS[q.get("kind", "shishkin")] for q in problems]
    rec["layer_cells"] = [int(q.get("layer_cells") or 0) for q in problems]
    rec["c"] = [c.ctypes.data for c, _ in keep]
    rec["r"] = [r.ctypes.data for _, r in keep]
    for f, n in zip(F, rec["N"].tolist()):
        if not (isinstance(f, torch.Tensor) and f.is_cuda and f.dtype == torch.float64
                and f.is_contiguous() and f.numel() == n - 1):
            raise TypeError("F must hold contiguous float64 device vectors of N-1 values")
    if U is None:  # views of one allocation
        sizes = [f.numel() for f in F]
        U = list(torch.split(torch.empty(sum(sizes), dtype=torch.float64, device=F[0].device), sizes))
    fa = np.array([f.data_ptr() for f in F], dtype=np.uint64)
    ua = np.array([u.data_ptr() for u in U], dtype=np.uint64)
    infos = np.zeros(S, dtype=np.dtype(Info1D))
    stream = torch.cuda.current_stream().cuda_stream
    rc = _check(lib().blp1d_solve(S, rec.ctypes.data_as(C.POINTER(Problem1D)),
                                  fa.ctypes.data_as(C.POINTER(C.c_void_p)),
                                  ua.ctypes.data_as(C.POINTER(C.c_void_p)),
                                  C.byref(Opts1D(maxit, int(left), K, g)), C.c_void_p(stream),
                                  infos.ctypes.data_as(C.POINTER(Info1D))), "blp1d_solve")
    del keep
    cols = [infos[k].tolist() for k, _ in Info1D._fields_]
    names = [k for k, _ in Info1D._fields_]
    out = [dict(zip(names, v), status=rc) for v in zip(*cols)]
    return U, out
