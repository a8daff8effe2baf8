"""GPU parity on other layer-adapted meshes: Bakhvalov-Shishkin graded layer
cells and Shishkin meshes with a quarter or three quarters of the cells in
the layer (Sec. 2.2's general construction; Sec. 3 admits any fitted tensor
mesh with a transition point).  The HIP path takes the mesh through
blp_mesh_opts; everything downstream (regions, lines, corner levels) follows
the transition index.  Same tolerances as the Shishkin parity tests:
operator applies 1e-14 of |A||x|, fixed-cycle preconditioner applies 1e-11,
FP64 solves equal iteration counts and corner cycles with error at most
1e-8 against the oracle's tight solution, mixed solves error at most 1e-6."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_13468_amd import inputs

pytestmark = pytest.mark.gpu

# (mesh kind, N, layer cells): interior widths of 3 to 12 bands, corners of
# 64 to 384 nodes (odd coarsest levels included), edge lines of 64 to 384 nodes
MESHES = [("bakhvalov-shishkin", 256, None), ("bakhvalov-shishkin", 512, 128),
          ("shishkin", 512, 128), ("shishkin", 512, 384), ("bakhvalov-shishkin", 1024, None)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pair(kind, N, nl, eps, seed, mg_fixed=0, prec=True):
    import torch
    assert torch.cuda.is_available()
    from paper_2108_13468_amd import blp
    inst = inputs.plain(N, eps, seed=seed)
    inst.mesh_kind, inst.layer_cells = kind, nl
    gp = blp.from_instance(inst)
    if prec:
        gp.precondition(mg_fixed=mg_fixed)
    op = O.Problem(N, eps, c1=inst.c1_at, c2=inst.c2_at, r=inst.r_const, mesh_kind=kind,
                   layer_cells=nl)
    x, y = gp.nodes()
    np.testing.assert_allclose(x, op.x, rtol=4e-16, atol=0)
    np.testing.assert_allclose(y, op.y, rtol=4e-16, atol=0)
    return inst, gp, op


def dev(v):
    import torch
    return torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("kind,N,nl", MESHES)
def test_operator_and_preconditioner_parity(kind, N, nl):
    say("mesh %s N=%d layer cells %s" % (kind, N, nl))
    inst, gp, op = pair(kind, N, nl, 1e-6, seed=N + 7, mg_fixed=2)
    rng = np.random.default_rng(N + 7)
    x = rng.standard_normal(op.n)
    absAx = np.abs(op.csr()) @ np.abs(x)
    for name, ref in (("A", op.A(x)), ("AT", op.AT(x))):
        err = np.abs(host(gp.apply(name, dev(x))) - ref).max() / absAx.max()
        assert err <= 1e-14, (name, err)
    b = rng.standard_normal(op.n)
    for name, tr in (("MINV", False), ("MINVT", True)):
        ref = op.M_inv(b, transpose=tr, mg_fixed=2)
        err = np.abs(host(gp.apply(name, dev(b))) - ref).max() / np.abs(ref).max()
        say("  %s rel err %.3e" % (name, err))
        assert err <= 1e-11, (name, err)


@pytest.mark.parametrize("kind,N,nl", [m for m in MESHES if m[1] <= 512])
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_solves_against_oracle(kind, N, nl, eps):
    inst, gp, op = pair(kind, N, nl, eps, seed=N + 8)
    F = O.sine_series(N, op.x, op.y, inst.a)
    u_t, st_t, _, _ = op.fgmres(F, tol=1e-10, scaled=True, maxit=1000)
    assert st_t == 0
    _, st, io, hist = op.fgmres(F, tol=1e-8, scaled=True, maxit=1000)
    assert st == 0
    Fd = dev(F)
    U, info, h = gp.solve(Fd, tol=1e-8, scaled=True, precision="fp64", maxit=1000, hist=True)
    d = info[0]
    err = np.abs(host(U) - u_t).max() / np.abs(u_t).max()
    say("%s N=%d nl=%s eps=%g: fp64 %d iterations (oracle %d), cycles %d..%d (oracle %d..%d), "
        "error %.2e" % (kind, N, nl, eps, d["iterations"], io.iterations, d["mg_cycles_min"],
                        d["mg_cycles_max"], io.mg_cycles_min, io.mg_cycles_max, err))
    assert d["converged"] and d["iterations"] == io.iterations
    assert (d["mg_cycles_min"], d["mg_cycles_max"]) == (io.mg_cycles_min, io.mg_cycles_max)
    k = d["iterations"]
    np.testing.assert_allclose(h[0][: k + 1], hist[: k + 1], rtol=1e-6)
    U10, i10 = gp.solve(Fd, tol=1e-10, scaled=True, precision="fp64", maxit=1000)
    assert np.abs(host(U10) - u_t).max() <= 1e-8 * np.abs(u_t).max()
    Um, im = gp.solve(Fd, tol=1e-8, scaled=True, precision="mixed", maxit=1000)
    errm = np.abs(host(Um) - u_t).max() / np.abs(u_t).max()
    say("  mixed %d iterations, error %.2e" % (im[0]["iterations"], errm))
    assert im[0]["converged"] and errm <= 1e-6
