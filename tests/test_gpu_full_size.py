"""GPU solves at the full workload sizes, in the launch configurations the
benchmark times.

* N = 1024, eps = 1e-6 (the headline problem): single FP64 and mixed solves
  against the oracle's solution at relative residual 1e-10: max-norm
  relative error at most 1e-8 (FP64) and 1e-6 (mixed);
* N = 2048, eps = 1e-6 (the multi-right-hand-side workload): a graphed,
  autotuned batch of two forward and two adjoint mixed solves.  The oracle
  cannot solve at this size within a test, so each result is checked by a
  property that holds at any size: the true residual of the scaled system,
  computed with the oracle's operator, meets the tolerance."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_13468_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle(inst):
    return O.Problem(inst.N, inst.eps, c1=inst.c1_at, c2=inst.c2_at, r=inst.r_const,
                     sigma=inst.sigma, clow_x=inst.clow[0], clow_y=inst.clow[1])


def test_headline_problem_against_oracle():
    import torch
    assert torch.cuda.is_available()
    from paper_2108_13468_amd import blp
    inst = inputs.headline_case(1e-6)
    say("headline problem N=%d eps=%g" % (inst.N, inst.eps))
    gp = blp.from_instance(inst).precondition()
    op = _oracle(inst)
    F = O.sine_series(inst.N, op.x, op.y, inst.a)
    u_t, st, _, _ = op.fgmres(F, tol=1e-10, scaled=True)
    assert st == 0
    Fd = torch.as_tensor(F, device="cuda")
    for prec, bound in (("fp64", 1e-8), ("mixed", 1e-6)):
        U, info = gp.solve(Fd, tol=1e-8, scaled=True, precision=prec)
        assert info[0]["converged"], info
        err = np.abs(U.cpu().numpy() - u_t).max() / np.abs(u_t).max()
        say("  %s: %d iterations, error %.2e" % (prec, info[0]["iterations"], err))
        assert err <= bound


def test_multi_rhs_workload_residuals():
    import torch
    assert torch.cuda.is_available()
    from paper_2108_13468_amd import blp
    inst, A = inputs.multi_rhs_case()
    say("multi-RHS workload N=%d eps=%g, 2 of %d right-hand sides" % (inst.N, inst.eps, len(A)))
    p = blp.from_instance(inst).precondition()
    op = _oracle(inst)
    d = np.sqrt(op.csr().diagonal())
    Fs = [O.sine_series(inst.N, op.x, op.y, A[k]) for k in range(2)]
    b = blp.Batch([p, p], graphs=True, autotune=True)
    tol = 1e-8
    # one scaled-residual check per result: ||D^-1/2 (F - A u)|| <= tol ||D^-1/2 F||
    # (plus a margin for the FP64 evaluation order of the two residuals)
    U, info = b.solve([torch.as_tensor(F, device="cuda") for F in Fs], tol=tol, precision="mixed")
    for k in range(2):
        assert info[k]["converged"], info[k]
        u = U[k].cpu().numpy()
        rel = np.linalg.norm((Fs[k] - op.A(u)) / d) / np.linalg.norm(Fs[k] / d)
        say("  forward %d: %d iterations, scaled residual %.2e" % (k, info[k]["iterations"], rel))
        assert rel <= tol * (1 + 1e-3)
    L, info = b.solve_adjoint([torch.as_tensor(F, device="cuda") for F in Fs], tol=tol,
                              precision="mixed")
    for k in range(2):
        assert info[k]["converged"], info[k]
        lam = L[k].cpu().numpy()
        rel = np.linalg.norm((Fs[k] - op.AT(lam)) / d) / np.linalg.norm(Fs[k] / d)
        say("  adjoint %d: %d iterations, scaled residual %.2e" % (k, info[k]["iterations"], rel))
        assert rel <= tol * (1 + 1e-3)
