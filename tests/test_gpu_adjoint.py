"""GPU adjoint: the torch.autograd.Function over blp_solve / blp_solve_adjoint.

* N = 32 against the oracle's dense adjoint (LU of A^T), with the gradient
  formulas written out on the oracle side (tolerance 1e-8 relative to the
  largest gradient entry: both sides solve to 1e-13 / exactly);
* the adjoint workload (N = 512, eps = 1e-4, 16 x 16 coefficients, 4 x 4 r
  controls) against central differences of J with h = 1e-6: J is quadratic in
  the coefficients, so there the difference quotient is exact up to the solve
  tolerance (relative 1e-5); in the r controls it carries an O(h^2) term
  (relative 1e-4);
* several right-hand sides with a shared R: the gradient is the sum of the
  single-right-hand-side gradients.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_13468_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(inst, tol=1e-13):
    import torch
    assert torch.cuda.is_available()
    from paper_2108_13468_amd.autograd import Solver
    return Solver(inst.N, inst.eps, inst.c1_at, inst.c2_at, sigma=inst.sigma, clow=inst.clow,
                  tol=tol)


def _J(solver, a, R, uobs):
    import torch
    U = solver(torch.as_tensor(a), torch.as_tensor(R))
    return 0.5 * float(((U - uobs) ** 2).sum())


def _grad(solver, a, R, uobs):
    import torch
    at = torch.tensor(a, requires_grad=True)
    Rt = torch.tensor(R, requires_grad=True)
    U = solver(at, Rt)
    J = 0.5 * ((U - uobs) ** 2).sum()
    J.backward()
    return at.grad.numpy(), Rt.grad.numpy(), float(J.detach())


def test_autograd_matches_dense_adjoint_N32():
    import torch
    N, eps = 32, 1e-4
    say("adjoint vs dense N=%d" % N)
    case = inputs.adjoint_case(N=N, eps=eps, K=4, m=4)
    inst = case.inst
    # oracle: dense solves and the gradient formulas
    x = O.mesh_axis(N, eps)[1]

    def orc(a, R):
        p = O.Problem(N, eps, c1=inst.c1_at, c2=inst.c2_at, r=O.bilinear(N, x, x, R))
        A = p.csr().toarray()
        return np.linalg.solve(A, O.sine_series(N, p.x, p.y, a)), A, p

    uref, _, _ = orc(case.a_ref, case.R_ref)
    uobs = uref + case.noise
    u, A, p = orc(inst.a, inst.r_ctrl)
    lam = np.linalg.solve(A.T, u - uobs)
    ga_ref = O.sine_project(N, p.x, p.y, lam, 4, 4)
    gR_ref = -O.bilinear_project(N, p.x, p.y, lam * u, 4)

    solver = _solver(inst)
    ga, gR, J = _grad(solver, inst.a, inst.r_ctrl, torch.as_tensor(uobs, device="cuda"))
    assert J == pytest.approx(0.5 * np.sum((u - uobs) ** 2), rel=1e-10)
    assert np.abs(ga - ga_ref).max() <= 1e-8 * np.abs(ga_ref).max()
    assert np.abs(gR - gR_ref).max() <= 1e-8 * np.abs(gR_ref).max()


def test_autograd_finite_differences_adjoint_workload():
    import torch
    case = inputs.adjoint_case()  # N = 512, eps = 1e-4, K = 16, m = 4
    inst = case.inst
    say("adjoint FD N=%d eps=%g K=%d" % (inst.N, inst.eps, inst.a.shape[0]))
    # relative residual 1e-12 (near the FP64 floor of this system): the
    # perturbation of J is ~1e-12 J, i.e. ~1e-6 relative in a quotient with h = 1e-6
    solver = _solver(inst, tol=1e-12)
    with torch.no_grad():
        uref = solver(torch.as_tensor(case.a_ref), torch.as_tensor(case.R_ref))
    uobs = uref + torch.as_tensor(case.noise, device="cuda")
    a, R = inst.a, inst.r_ctrl
    ga, gR, J0 = _grad(solver, a, R, uobs)
    h = 1e-6
    for (l, k) in [(0, 0), (3, 7), (15, 15)]:
        ap, am = a.copy(), a.copy()
        ap[l, k] += h
        am[l, k] -= h
        fd = (_J(solver, ap, R, uobs) - _J(solver, am, R, uobs)) / (2 * h)
        say("  a[%d,%d]: adjoint %.10e fd %.10e" % (l, k, ga[l, k], fd))
        assert ga[l, k] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(ga).max())
    for (q, pp) in [(0, 0), (1, 2), (3, 3)]:
        Rp, Rm = R.copy(), R.copy()
        Rp[q, pp] += h
        Rm[q, pp] -= h
        fd = (_J(solver, a, Rp, uobs) - _J(solver, a, Rm, uobs)) / (2 * h)
        say("  R[%d,%d]: adjoint %.10e fd %.10e" % (q, pp, gR[q, pp], fd))
        assert gR[q, pp] == pytest.approx(fd, rel=1e-4, abs=1e-6 * np.abs(gR).max())


def test_autograd_several_right_hand_sides():
    import torch
    N, eps = 64, 1e-3
    say("adjoint nrhs=3 N=%d" % N)
    rng = np.random.default_rng(21)
    a3 = rng.uniform(-1, 1, size=(3, 4, 4))
    R = rng.uniform(0.5, 2.0, size=(4, 4))
    inst = inputs.Instance(N=N, eps=eps, r_const=None, r_ctrl=R, a=a3[0])
    solver = _solver(inst)
    uobs = torch.as_tensor(rng.standard_normal((3, (N - 1) ** 2)) * 1e-3, device="cuda")
    ga, gR, _ = _grad(solver, a3, R, uobs)
    gR_sum = np.zeros_like(R)
    for s in range(3):
        ga1, gR1, _ = _grad(solver, a3[s], R, uobs[s])
        assert np.abs(ga[s] - ga1).max() <= 1e-9 * np.abs(ga1).max()
        gR_sum += gR1
    assert np.abs(gR - gR_sum).max() <= 1e-9 * np.abs(gR_sum).max()


@pytest.mark.parametrize("m", [4, 5])
def test_reaction_gradient_entry_point(m):
    """blp_reaction_gradient: -sum over three stacked (lambda, u) pairs of the
    bilinear projection of lambda u (Sec. 3's reaction term enters A only on
    the diagonal), against the oracle's projection of each product."""
    import torch
    from paper_2108_13468_amd import blp
    N, eps = 96, 1e-4
    inst = inputs.plain(N, eps, seed=23)
    p = blp.from_instance(inst)
    x, y = p.nodes()
    rng = np.random.default_rng(24)
    lam = rng.standard_normal((3, (N - 1) ** 2))
    u = rng.standard_normal((3, (N - 1) ** 2))
    G = p.reaction_gradient(torch.as_tensor(lam, device="cuda"), torch.as_tensor(u, device="cuda"), m)
    ref = -sum(O.bilinear_project(N, x, y, lam[s] * u[s], m) for s in range(3))
    say("reaction gradient m=%d: max |G - ref| = %.2e" % (m, np.abs(G - ref).max()))
    assert np.abs(G - ref).max() <= 1e-12 * np.abs(ref).max()
