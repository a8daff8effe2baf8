"""torch.autograd.Function through the library's solve and adjoint solve.

The map (a, R) -> U: sine-series coefficients a of the forcing (L x K, or
nrhs x L x K for several right-hand sides) and the bilinear controls R of the
reaction field (m x m, shared) give U = A(R)^{-1} F(a), the discrete solution
on the interior nodes.  For a scalar J(U) the backward pass uses the discrete
adjoint:
  A^T lambda = dJ/dU          (blp_solve_adjoint: FGMRES with M^T),
  dJ/da_kl = sum_ij lambda_ij sin(k pi x_i) sin(l pi y_j)   (blp_sine_project),
  dJ/dR_pq = -sum_ij lambda_ij u_ij phi_p(x_i) phi_q(y_j)   (blp_reaction_gradient),
since F is linear in a and A depends on r only through its diagonal, with r
the bilinear interpolant of R on control nodes {0, 1/(m-1), ..., 1} in each
axis.  The mesh depends on eps, N and the convection bounds only, so neither
gradient has a mesh term.  Every step runs in the library; this module only
moves arguments.
"""
import numpy as np
import torch

from . import blp


class Solver:
    """Fixed problem data (N, eps, convection, mesh parameters, solve options)
    for SolveFunction.  c1, c2: callables of the node coordinate or arrays of
    the N+1 nodal values.  The assembled and preconditioned problem is cached
    for the last R seen."""

    def __init__(self, N, eps, c1, c2, sigma=2.0, clow=(1.0, 1.0), tol=1e-12, scaled=True,
                 precision="fp64", restart=50, maxit=2000, mg_fixed=0):
        self.N, self.eps, self.sigma, self.clow = N, eps, sigma, tuple(clow)
        _, x, y = blp.mesh(N, eps, sigma, self.clow)
        self.c1 = np.asarray(c1(x) if callable(c1) else c1, dtype=np.float64)
        self.c2 = np.asarray(c2(y) if callable(c2) else c2, dtype=np.float64)
        self.opts = dict(tol=tol, scaled=scaled, precision=precision, restart=restart, maxit=maxit)
        self.mg_fixed = mg_fixed
        self._key = None
        self._p = None
        self.last_info = None

    def problem(self, R):
        R = np.ascontiguousarray(R, dtype=np.float64)
        key = (R.shape, R.tobytes())
        if key != self._key:
            self._p = blp.Problem(self.N, self.eps, ("axis", self.c1), ("axis", self.c2),
                                  ("bilinear", R), sigma=self.sigma, clow=self.clow)
            self._p.precondition(mg_fixed=self.mg_fixed)
            self._key = key
        return self._p

    def __call__(self, a, R):
        return SolveFunction.apply(a, R, self)


def _require_converged(info, what):
    bad = [k for k, d in enumerate(info) if not d["converged"]]
    if bad:
        raise blp.BlpError("%s did not converge for right-hand side(s) %s" % (what, bad))


class SolveFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, R, solver):
        an = a.detach().cpu().to(torch.float64).numpy()
        Rn = R.detach().cpu().to(torch.float64).numpy()
        p = solver.problem(Rn)
        a3 = an if an.ndim == 3 else an[None]
        nrhs = a3.shape[0]
        F = torch.empty((nrhs, p.n), dtype=torch.float64, device=p.device)
        for s in range(nrhs):
            p.sine_rhs(a3[s], out=F[s])
        U, info = p.solve(F.reshape(-1), **solver.opts)
        _require_converged(info, "forward solve")
        solver.last_info = info
        U = U.reshape(nrhs, p.n)
        ctx.p, ctx.solver = p, solver
        ctx.a_shape, ctx.R_shape = an.shape, Rn.shape
        ctx.a_meta, ctx.R_meta = (a.device, a.dtype), (R.device, R.dtype)
        ctx.save_for_backward(U)
        return U if an.ndim == 3 else U[0]

    @staticmethod
    def backward(ctx, gU):
        (U,) = ctx.saved_tensors
        p = ctx.p
        nrhs = U.shape[0]
        G = gU.detach().to(torch.float64).reshape(nrhs, p.n).contiguous()
        lam, info = p.solve_adjoint(G.reshape(-1), **ctx.solver.opts)
        _require_converged(info, "adjoint solve")
        lam = lam.reshape(nrhs, p.n)
        L, K = ctx.a_shape[-2:]
        ga = np.stack([p.sine_project(lam[s], K, L) for s in range(nrhs)])
        gR = None
        if ctx.needs_input_grad[1]:
            # summed over the right-hand sides, sign included, on the device
            gR = p.reaction_gradient(lam, U, ctx.R_shape[0])
        ga_t = torch.from_numpy(ga.reshape(ctx.a_shape)).to(*ctx.a_meta)
        gR_t = None if gR is None else torch.from_numpy(gR).to(*ctx.R_meta)
        return ga_t, gR_t, None
