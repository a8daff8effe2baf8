"""GPU batched solves (blp_batch_*, and blp_solve with several right-hand
sides): each system of a batch follows exactly the iteration of its single
solve (same restart cycles, same kernels on the same data), so the batched
result equals the single-solve result up to rounding (asserted to 1e-13
relative, with equal iteration counts); one mixed-precision batch of the
uneven-batch recipe is also checked against the oracle (the mixed target,
1e-6 max-norm relative error)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_13468_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problems(insts, mg_fixed=0):
    import torch
    assert torch.cuda.is_available()
    from paper_2108_13468_amd import blp
    ps = [blp.from_instance(i).precondition(mg_fixed=mg_fixed) for i in insts]
    return ps, [p.sine_rhs(i.a) for p, i in zip(ps, insts)]


def _rel(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("precision,graphs,tune", [("fp64", False, False), ("mixed", False, False),
                                                   ("fp64", True, False), ("mixed", True, True)])
def test_batch_matches_single_solves(precision, graphs, tune):
    """With graphs, every Krylov step replays the two captured graphs of each
    mesh size (eager launches, memcpys and host decisions in between): each
    replay must reproduce the eager single solve."""
    from paper_2108_13468_amd import blp
    insts = inputs.batch_cases(count=6, seed=31, sizes=(64, 96, 130))
    say("batch of %d, sizes %s, %s, graphs=%s, autotune=%s" % (
        len(insts), [i.N for i in insts], precision, graphs, tune))
    ps, F = _problems(insts)
    opts = dict(tol=1e-10, scaled=True, precision=precision, maxit=800)
    single = [p.solve(f, **opts) for p, f in zip(ps, F)]
    b = blp.Batch(ps, graphs=graphs, autotune=tune)
    for rep in range(2):  # the second solve replays graphs captured by the first
        U, info = b.solve(F, **opts)
        for s in range(len(ps)):
            assert info[s]["converged"] == 1
            assert info[s]["iterations"] == single[s][1][0]["iterations"], (rep, s)
            # identical schedules agree to rounding; a tuned line-solve variant
            # groups its scans differently (other rounding in the preconditioner),
            # which moves the result well inside the solve tolerance
            assert _rel(U[s], single[s][0]) <= (1e-9 if tune else 1e-13), (rep, s)
    if tune:
        say(b.describe())


def test_batch_adjoint_matches_single():
    from paper_2108_13468_amd import blp
    insts = inputs.batch_cases(count=4, seed=32, sizes=(64, 128))
    say("adjoint batch sizes %s" % [i.N for i in insts])
    ps, F = _problems(insts)
    single = [p.solve_adjoint(f, tol=1e-10) for p, f in zip(ps, F)]
    L, info = blp.Batch(ps).solve_adjoint(F, tol=1e-10)
    for s in range(len(ps)):
        assert info[s]["iterations"] == single[s][1][0]["iterations"], s
        assert _rel(L[s], single[s][0]) <= 1e-13, s


def test_several_right_hand_sides_match_single():
    import torch
    inst = inputs.plain(96, 1e-5, seed=33)
    ps, _ = _problems([inst])
    p = ps[0]
    rng = np.random.default_rng(33)
    F = torch.stack([p.sine_rhs(rng.uniform(-1, 1, size=(3, 3))) for _ in range(3)])
    say("nrhs=3 N=96")
    U, info = p.solve(F.reshape(-1), tol=1e-10)
    U = U.reshape(3, -1)
    for k in range(3):
        u1, i1 = p.solve(F[k].contiguous(), tol=1e-10)
        assert info[k]["iterations"] == i1[0]["iterations"]
        assert _rel(U[k], u1) <= 1e-13


def test_mixed_batch_against_oracle():
    from paper_2108_13468_amd import blp
    insts = inputs.batch_cases(count=5, seed=34, sizes=(64, 128))
    say("mixed batch vs oracle, sizes %s eps %s" % ([i.N for i in insts],
                                                   ["%.1e" % i.eps for i in insts]))
    ps, F = _problems(insts)
    U, info = blp.Batch(ps).solve(F, tol=1e-8, precision="mixed", maxit=800)
    for s, inst in enumerate(insts):
        assert info[s]["converged"] == 1
        op = O.Problem(inst.N, inst.eps, c1=inst.c1_at, c2=inst.c2_at, r=inst.r_const)
        # reference at scaled relative residual 1e-9 (the FP64 floor at eps ~ 1e-8
        # lies near 1e-10; the error of the reference stays far below 1e-6)
        ue, st, _, _ = op.fgmres(O.sine_series(inst.N, op.x, op.y, inst.a), tol=1e-9,
                                 scaled=True, maxit=2000)
        assert st == 0
        err = np.abs(U[s].cpu().numpy() - ue).max() / np.abs(ue).max()
        say("  system %d N=%d eps=%.1e it=%d err %.2e" % (s, inst.N, inst.eps,
                                                         info[s]["iterations"], err))
        assert err <= 1e-6


def test_alternating_precisions_reuse_plans():
    """Solves that alternate FP64 and mixed precision on one problem, with a
    fresh result vector each time, reuse their plans (rebound to the new
    vectors) and the per-precision Krylov workspaces: every repeat reproduces
    the first solve of its precision bit for bit, with the same iterations."""
    inst = inputs.plain(256, 1e-5, seed=7)
    say("alternating precisions N=%d" % inst.N)
    (p,), (F,) = _problems([inst])
    first = {}
    for rnd in range(3):
        for prec in ("fp64", "mixed"):
            U, info = p.solve(F, tol=1e-8, scaled=True, precision=prec)
            it = info[0]["iterations"]
            assert info[0]["converged"]
            if rnd == 0:
                first[prec] = (U.clone(), it)
            else:
                U0, it0 = first[prec]
                assert it == it0
                assert bool((U == U0).all()), (prec, rnd, _rel(U, U0))


def test_full_batch_recipe_against_references():
    """The 64-instance uneven batch exactly as the benchmark runs it (graphs,
    autotuner, mixed precision, scaled relative residual 1e-8), compared with
    references for the instances that set its difficulty: the two with the
    most iterations (N = 1024 at eps near 5e-4, N = 512 at eps near 2e-3),
    the smallest eps of each mesh size (down to 1.2e-8), and the largest eps
    at N = 128 and 256.  References: for eps >= 1e-4, where restarted FGMRES
    needs hundreds of iterations, the direct solve of the oracle's matrix;
    below, the oracle's FGMRES to a scaled relative residual of 1e-9 (a few
    iterations; the FP64 floor of both there lies near 1e-10).  Bound: the
    mixed target, 1e-6 max-norm relative error; every instance of the batch
    must converge."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2108_13468_amd import blp
    from tests.reference import direct, max_rel
    insts = inputs.batch_cases(64)
    picks = [13, 47, 10, 61, 15, 16, 41, 58]
    say("full batch recipe: references for instances %s (N %s, eps %s)" % (
        picks, [insts[k].N for k in picks], ["%.1e" % insts[k].eps for k in picks]))

    def ref(k):
        i = insts[k]
        op = O.Problem(i.N, i.eps, c1=i.c1_at, c2=i.c2_at, r=i.r_const)
        F = O.sine_series(i.N, op.x, op.y, i.a)
        if i.eps >= 1e-4:
            return direct(op, F)
        u, st, io, _ = op.fgmres(F, tol=1e-9, scaled=True, maxit=500)
        assert st == 0
        return u, io.true_res / io.norm_F

    slow = [k for k in picks if insts[k].eps >= 1e-4 and insts[k].N >= 512]
    with ThreadPoolExecutor(2) as ex:
        # the large direct solves one at a time, the rest beside them
        futs_slow = ex.submit(lambda: {k: ref(k) for k in slow})
        futs_fast = ex.submit(lambda: {k: ref(k) for k in picks if k not in slow})
        ps, F = _problems(insts)
        b = blp.Batch(ps, graphs=True, autotune=True)
        U, info = b.solve(F, tol=1e-8, precision="mixed", maxit=2000)
        torch.cuda.synchronize()
        refs = dict(futs_slow.result())
        refs.update(futs_fast.result())
    assert all(d["converged"] == 1 for d in info), [k for k, d in enumerate(info)
                                                     if not d["converged"]]
    it = [d["iterations"] for d in info]
    say("  iterations: max %d, mean %.1f" % (max(it), float(np.mean(it))))
    for k in picks:
        u_t, res = refs[k]
        assert res <= 1e-9, (k, res)
        err = max_rel(U[k].cpu().numpy(), u_t)
        say("  instance %d N=%d eps=%.2e: %d iterations, error %.2e (reference residual %.1e)" % (
            k, insts[k].N, insts[k].eps, it[k], err, res))
        assert err <= 1e-6, k
