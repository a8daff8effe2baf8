"""GPU parity of the one-dimensional method (Sec. 2, blp1d_solve): every
problem of a batch runs unrestarted GMRES with M of eq. block_M inside one
launch, one workgroup per problem.

* Table 2 in one launch: the 26 printed (eps, N) cases of the paper's test
  problem (c = 2 + sin 5x, r = 1, f = 4 exp(-x), Clow = 0.99), M on the left,
  stopped at ||F - A u||_inf <= K ln(N)/N with K = ||U^E||_inf computed on
  the device: every printed count, the oracle's counts, the oracle's K to
  1e-12 and its iterates to 1e-10 (same algorithm; the GPU's tridiagonal
  solves are scans, so they differ by rounding only).
* M on the right and on the left, uneven sizes (N = 4 to 4096), other layer
  meshes and random coefficients: equal counts and iterates against the
  oracle (1e-10 on the left, 1e-7 on the right, where the iterate ends with
  an M^{-1} apply whose rounding the condition of M amplifies).
* maxit reached: BLP_W_NOCONV with the record filled in; bad arguments:
  BLP_E_INVAL."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
CLOW = 0.99


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def c_fun(x):
    return 2.0 + np.sin(5.0 * x)


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            e, n, v = line.split()
            out[(float(e), int(n))] = float(v)
    return out


def case(N, eps, c=c_fun, r=1.0, f=lambda x: 4.0 * np.exp(-x), kind="shishkin", nl=None,
         sigma=2.0, clow=CLOW):
    """(oracle problem, GPU problem, F): each side evaluates c, r and f at the
    nodes of its own mesh code (the two meshes agree to rounding)."""
    from paper_2108_13468_amd import blp
    p = O.Problem1D(N, eps, c, r, sigma=sigma, clow=clow, mesh_kind=kind, layer_cells=nl)
    _, x, _ = blp.mesh(N, eps, sigma, (clow, clow), kind, nl)
    np.testing.assert_allclose(x, p.x, rtol=4e-16, atol=0)
    q = dict(N=N, eps=eps, c=c(x), r=np.full(N + 1, float(r)), sigma=sigma, clow=clow, kind=kind,
             layer_cells=nl, F=f(x[1:-1]))
    return p, q, f(p.x[1:-1])


def run(cases, **kw):
    import torch
    assert torch.cuda.is_available()
    from paper_2108_13468_amd import blp
    F = [torch.as_tensor(q["F"], device="cuda") for _, q, _ in cases]
    U, info = blp.solve_1d([q for _, q, _ in cases], F, **kw)
    return [u.cpu().numpy() for u in U], info


def test_table2_in_one_launch():
    ref = read_golden("table2_1d_iterations.txt")
    keys = sorted(ref)
    cases = [case(N, eps) for eps, N in keys]
    U, info = run(cases, maxit=100, left=True)
    for (eps, N), (p, q, F), u, d in zip(keys, cases, U, info):
        UE = p.solve(F)
        K = np.abs(UE).max()
        uo, st, io, _ = p.gmres(F, K=K, g=np.log(N) / N, maxit=100, left=True)
        diff = np.abs(u - uo).max() / np.abs(uo).max()
        say("eps=%g N=%d: %d iterations (Table 2: %d, oracle %d), K %.6e, iterate diff %.1e" % (
            eps, N, d["iterations"], ref[(eps, N)], io.iterations, d["K"], diff))
        assert d["converged"] and d["iterations"] == int(ref[(eps, N)]) == io.iterations
        assert d["K"] == pytest.approx(K, rel=1e-12)
        assert diff <= 1e-10
        assert d["res_inf"] <= K * np.log(N) / N


def test_right_preconditioning_uneven_meshes_and_coefficients():
    rng = np.random.default_rng(9)
    specs = [(4, 1e-1, "shishkin", None), (16, 1e-3, "shishkin", None),
             (256, 1e-5, "bakhvalov-shishkin", None), (512, 1e-6, "shishkin", 128),
             (1000, 1e-4, "shishkin", 300), (2048, 1e-7, "bakhvalov-shishkin", 512),
             (4096, 1e-8, "shishkin", None)]
    cases = []
    for N, eps, kind, nl in specs:
        a, b = rng.uniform(0.5, 1.0), rng.uniform(0.0, 2.0)
        cases.append(case(N, eps, c=lambda x, a=a: 1.0 + a * x, r=b,
                          f=lambda x, s=rng.uniform(1, 3): np.sin(s * np.pi * x) + 1.0,
                          kind=kind, nl=nl, clow=1.0))
    for left in (False, True):
        U, info = run(cases, maxit=120, left=left)
        for (N, eps, kind, nl), (p, q, F), u, d in zip(specs, cases, U, info):
            K = np.abs(p.solve(F)).max()
            uo, st, io, _ = p.gmres(F, K=K, g=np.log(N) / N, maxit=120, left=left)
            diff = np.abs(u - uo).max() / np.abs(uo).max()
            say("%s N=%d eps=%g %s nl=%s: %d iterations (oracle %d), diff %.1e" % (
                "left" if left else "right", N, eps, kind, nl, d["iterations"], io.iterations, diff))
            assert d["iterations"] == io.iterations and d["converged"] == io.converged
            # the right-preconditioned iterate ends with an M^{-1} apply; its two
            # evaluation orders (sequential Thomas, scans) differ by rounding
            # amplified by the condition of M, which grows like 1/(eps N) (seen:
            # 2.5e-10 at eps = 1e-7, N = 2048; 7.6e-9 at eps = 1e-8, N = 4096)
            assert diff <= (1e-10 if left else 1e-7)


def test_cap_and_argument_errors():
    import torch
    from paper_2108_13468_amd import blp
    p, q, F = case(2048, 1e-4)
    U, info = run([(p, q, F)], maxit=3, left=True)
    assert info[0]["status"] == 1 and info[0]["iterations"] == 3 and not info[0]["converged"]
    assert np.isfinite(info[0]["res_inf"]) and info[0]["res_inf"] > 0
    bad = dict(q)
    bad["N"] = 63
    with pytest.raises(blp.BlpError) as e:
        blp.solve_1d([bad], [torch.zeros(62, dtype=torch.float64, device="cuda")])
    assert e.value.code == -1
    bad = dict(q)
    bad["c"] = -bad["c"]
    with pytest.raises(blp.BlpError) as e:
        blp.solve_1d([bad], [torch.as_tensor(q["F"], device="cuda")])
    assert e.value.code == -1
