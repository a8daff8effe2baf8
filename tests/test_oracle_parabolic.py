"""Pins of the oracle's case with one parabolic and one exponential layer
(Sec. 3: c2 = 0, eq. tau parabolic; Sec. 3.2: corner multigrid with
x-semicoarsening; Sec. 3.3: eq. parabolic_MMS, Tables 3 and 4).

None of these retypes the oracle's formulas.  They check what fixes them
from outside:
* the transition point of the parabolic axis (closed form, uniform limit);
* the interpolation by its defining property (an interpolated vector solves
  every odd node's North-South-collapsed row; even nodes are injected);
* restriction = P^T and the Galerkin coarse operator = P^T A P, both
  against scipy sparse products built from the interpolation's action;
* the closed-form coarse stencil of a pure-diffusion operator on a uniform
  grid (linear interpolation, mass-lumped y-part);
* a Gauss-Seidel sweep = a triangular solve in the downstream ordering;
* many cycles = the exact corner solve (banded LU);
* the paper's printed numbers: all 20 errors of Table 3, all 20 iteration
  counts of Table 4 and the three cycles per corner solve.

Reading pinned here (as in the one-dimensional tables): the x-layer mesh
takes the lower bound Clow = 0.99 of c1 = 1; with Clow = 1 the errors come
out 0.8% lower.  The iteration counts use the estimate stopping test of
Sec. 3.3 (the same reading that reproduces Table 7)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_2108_13468_amd import inputs
from tests.mms import parabolic_mms

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            e, n, v = line.split()
            out[(float(e), int(n))] = float(v)
    return out


def problem(N, eps, **kw):
    inst = inputs.mms_parabolic(N, eps)
    args = dict(c1=inst.c1_at, c2=inst.c2_at, r=inst.r_const, sigma=inst.sigma,
                clow_x=inst.clow[0], clow_y=inst.clow[1], y_layer=inst.y_layer)
    args.update(kw)
    return O.Problem(N, eps, **args)


def random_problem(N, eps, seed=0, uniform=False):
    """Variable c1(x), c2 = 0, random positive r(x, y)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.5, 2.0, size=(N - 1) ** 2)
    return O.Problem(N, eps, c1=lambda x: 1.0 + x ** 2, c2=np.zeros(N + 1), r=r,
                     sigma=2.5, y_layer="parabolic")


def level_matrix(p, l):
    """Sparse matrix of level l from its exported 9-point stencils."""
    a = p.par_stencil(l)
    ny, nx = a.shape[:2]
    rows, cols, vals = [], [], []
    for j in range(ny):
        for i in range(nx):
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    v = a[j, i, dj + 1, di + 1]
                    if v != 0.0:
                        rows.append(j * nx + i)
                        cols.append((j + dj) * nx + (i + di))
                        vals.append(v)
    n = nx * ny
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def interp_matrix(p, l):
    """P from level l+1 to level l, column by column from its action."""
    nf, nc, ny = p.par_levels[l], p.par_levels[l + 1], p.h
    cols = []
    for k in range(nc * ny):
        e = np.zeros(nc * ny)
        e[k] = 1.0
        cols.append(sp.csr_matrix(p.par_op("interp", l, e)).T)
    return sp.hstack(cols).tocsr()


# --------------------------------------------------------------- mesh ----

@pytest.mark.parametrize("N,eps", [(128, 1e-5), (512, 1e-8), (2048, 1e-6), (128, 1e-2)])
def test_parabolic_transition_point(N, eps):
    """eq. tau parabolic: tau_y = min(1/2, sigma sqrt(eps) ln N), N/2 equal
    cells on each side; tau_x keeps the exponential form with Clow; the y
    mesh does not depend on the y lower bound."""
    p = problem(N, eps)
    assert p.tau_y == pytest.approx(min(0.5, 2.5 * np.sqrt(eps) * np.log(N)), rel=1e-15)
    assert p.tau_x == pytest.approx(min(0.5, 2.5 * eps * np.log(N) / 0.99), rel=1e-15)
    h = N // 2
    np.testing.assert_allclose(np.diff(p.y[: h + 1]), p.tau_y / h, rtol=1e-12)
    np.testing.assert_allclose(np.diff(p.y[h:]), (1 - p.tau_y) / h, rtol=1e-12)
    q = problem(N, eps, clow_y=0.3)
    np.testing.assert_array_equal(q.y, p.y)
    if eps == 1e-2:  # sigma sqrt(eps) ln N > 1/2: the uniform mesh
        np.testing.assert_allclose(np.diff(p.y), 1.0 / N, rtol=1e-12)


# ------------------------------------------------------ the hierarchy ----

def test_semicoarsening_levels():
    """Coarsening by two in x only, down to two columns; every level keeps
    all h rows."""
    p = random_problem(64, 1e-6)
    assert p.par_levels == [32, 16, 8, 4, 2]
    p = random_problem(48, 1e-6)  # h = 24: 24, 12, 6, 3 (odd: stop)
    assert p.par_levels == [24, 12, 6, 3]


@pytest.mark.parametrize("eps", [1e-3, 1e-7])
def test_interpolation_solves_collapsed_rows(eps):
    """Operator-induced interpolation (Sec. 3.2): P v is v at the even
    nodes, and at every odd node it satisfies that node's row of the level
    operator with the rows j-1, j, j+1 collapsed onto row j (homogeneous
    equation), on every level."""
    p = random_problem(64, eps, seed=1)
    rng = np.random.default_rng(2)
    for l in range(len(p.par_levels) - 1):
        nf, nc, ny = p.par_levels[l], p.par_levels[l + 1], p.h
        v = rng.standard_normal(nc * ny)
        z = p.par_op("interp", l, v).reshape(ny, nf)
        V = v.reshape(ny, nc)
        np.testing.assert_array_equal(z[:, 1::2], V)  # even i (1-based) = odd index
        a = p.par_stencil(l).sum(axis=2)  # [j, i, di+1]: collapsed over dj
        zp = np.pad(z, ((0, 0), (1, 1)))
        for i in range(1, nf + 1, 2):  # odd fine nodes
            res = a[:, i - 1, 0] * zp[:, i - 1] + a[:, i - 1, 1] * zp[:, i] + a[:, i - 1, 2] * zp[:, i + 1]
            scale = (np.abs(a[:, i - 1, :]) * np.abs(zp[:, i - 1:i + 2])).sum(axis=1)
            assert np.all(np.abs(res) <= 1e-13 * scale), (l, i)


@pytest.mark.parametrize("eps", [1e-2, 1e-6])
def test_galerkin_coarse_operators(eps):
    """Every coarse level is P^T A P of the level above (9-point), and
    restriction is P^T, with P taken from the interpolation's action."""
    p = random_problem(32, eps, seed=3)
    for l in range(len(p.par_levels) - 1):
        A = level_matrix(p, l)
        P = interp_matrix(p, l)
        Ac = level_matrix(p, l + 1)
        G = (P.T @ A @ P).toarray()
        np.testing.assert_allclose(Ac.toarray(), G, rtol=0, atol=1e-13 * np.abs(G).max())
        r = np.random.default_rng(l).standard_normal(A.shape[0])
        np.testing.assert_allclose(p.par_op("restrict", l, r), P.T @ r, rtol=1e-13, atol=1e-15)
        # the 9-point pattern closes: no coupling beyond one coarse node
        assert Ac.nnz <= 9 * Ac.shape[0]


def test_finest_level_is_the_rescaled_corner_block():
    """Level 0 = diag(hbar_i kbar_j) A_CC, A_CC the corner block of A."""
    p = random_problem(32, 1e-5, seed=4)
    h, n1 = p.h, p.n1
    A = p.csr()
    idx = np.array([(j - 1) * n1 + (i - 1) for j in range(1, h + 1) for i in range(1, h + 1)])
    Acc = A[idx][:, idx].toarray()
    hb = 0.5 * (p.hx[1:h + 1] + p.hx[2:h + 2])
    kb = 0.5 * (p.hy[1:h + 1] + p.hy[2:h + 2])
    S = np.outer(kb, hb).ravel()
    np.testing.assert_allclose(level_matrix(p, 0).toarray(), S[:, None] * Acc, rtol=1e-15,
                               atol=0)


def test_pure_diffusion_closed_form():
    """-Lap on a uniform grid (c = 0, r = 0, eps = 1, so both transition
    points are 1/2): FE rescaling gives the stencil eps [-1; -1 4 -1; -1];
    away from the top and bottom rows the interpolation is linear (weights
    1/2), and the Galerkin coarse operator is the x-stiffness on the coarse
    x-mesh plus the y-stiffness times P^T P = [1/4 3/2 1/4] in x:
      centre 4, (+-1, 0) 0, (0, +-1) -3/2, (+-1, +-1) -1/4."""
    N = 32
    p = O.Problem(N, 1.0, c1=np.zeros(N + 1), c2=np.zeros(N + 1), r=0.0, sigma=2.5,
                  y_layer="parabolic")
    np.testing.assert_allclose(np.diff(p.x), 1.0 / N, rtol=1e-12)
    np.testing.assert_allclose(np.diff(p.y), 1.0 / N, rtol=1e-12)
    a0 = p.par_stencil(0)
    np.testing.assert_allclose(a0[5, 5], [[0, -1, 0], [-1, 4, -1], [0, -1, 0]], rtol=1e-13,
                               atol=1e-15)
    wl, wr = p.par_weights(0)
    np.testing.assert_allclose(wl[1:-1, 2::2], 0.5, rtol=1e-14)  # node 1: no left coarse node
    assert np.all(wl[:, 0] == 0.0)
    np.testing.assert_allclose(wr[1:-1, 0::2], 0.5, rtol=1e-14)
    a1 = p.par_stencil(1)
    nc = p.par_levels[1]
    expect = np.array([[-0.25, -1.5, -0.25], [0.0, 4.0, 0.0], [-0.25, -1.5, -0.25]])
    for J in range(3, p.h - 2 + 1):
        for I in range(2, nc):
            np.testing.assert_allclose(a1[J - 1, I - 1], expect, rtol=0, atol=1e-13)


# ------------------------------------------------------------ cycling ----

def test_gauss_seidel_is_downstream_triangular_solve():
    """One sweep = (D + U)^{-1} (b - L z): nodes later in the natural order
    (higher rows, further right) are updated first, so their new values
    enter (U, including the North-West coupling of a 9-point level)."""
    p = random_problem(32, 1e-6, seed=5)
    rng = np.random.default_rng(6)
    for l in (0, 1, len(p.par_levels) - 1):
        A = level_matrix(p, l).toarray()
        n = A.shape[0]
        b, z = rng.standard_normal(n), rng.standard_normal(n)
        got = p.par_op("gs", l, b, z)
        want = np.linalg.solve(np.triu(A), b - np.tril(A, -1) @ z)
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("N,eps", [(64, 1e-4), (128, 1e-8)])
def test_cycles_converge_to_the_exact_corner_solve(N, eps):
    p = random_problem(N, eps, seed=7)
    b = np.random.default_rng(8).standard_normal(p.h ** 2)
    z, cyc = p.corner_mg(b, fixed=40)
    ze = p.corner_exact(b)
    assert cyc == 40
    assert np.abs(z - ze).max() <= 1e-11 * np.abs(ze).max()
    # the adaptive rule: reduction of the rescaled residual by 1e2
    z2, cyc2 = p.corner_mg(b, rtol=1e-2)
    assert 1 <= cyc2 <= 5


def test_no_transposed_parabolic_cycle():
    p = random_problem(16, 1e-4)
    with pytest.raises(ValueError):
        p.corner_mg(np.ones(p.h ** 2), transpose=True)
    z = p.M_inv(np.ones(p.n), transpose=True)
    assert np.isnan(z).any()


# ------------------------------------------------------ Tables 3 and 4 ----

def table_case(N, eps):
    p = problem(N, eps)
    u, f = parabolic_mms(eps, p.x, p.y)
    U, st, info, _ = p.fgmres(f, tol=10 * np.log(N) / N, absolute=True, mg_rtol=1e-2,
                              stop_on_estimate=True)
    assert st == 0
    return np.abs(U - u).max(), info


@pytest.mark.parametrize("eps", [1e-5, 1e-6, 1e-7, 1e-8])
def test_tables_3_and_4(eps):
    """Sec. 3.3 (sigma = 5/2, ||R||_2 <= 10 ln N / N, corner cycles to a 1e2
    reduction): the errors of Table 3 to the printed digits, the iteration
    counts of Table 4, and three V-cycles per corner solve, N = 128 to
    1024."""
    errs = read_golden("table3_parabolic_errors.txt")
    its = read_golden("table4_parabolic_iterations.txt")
    for N in (128, 256, 512, 1024):
        err, info = table_case(N, eps)
        assert err == pytest.approx(errs[(eps, N)], rel=6e-4), (N, err)
        assert info.iterations == int(its[(eps, N)]), (N, info.iterations)
        assert info.mg_cycles_min == info.mg_cycles_max == 3


def test_tables_3_and_4_at_2048():
    """The N = 2048 column: errors and counts as printed; the corner solves
    take two or three cycles (two where the top layer is widest)."""
    errs = read_golden("table3_parabolic_errors.txt")
    its = read_golden("table4_parabolic_iterations.txt")
    for eps in (1e-5, 1e-6, 1e-7, 1e-8):
        err, info = table_case(2048, eps)
        assert err == pytest.approx(errs[(eps, 2048)], rel=6e-4), (eps, err)
        assert info.iterations == int(its[(eps, 2048)]), (eps, info.iterations)
        assert 2 <= info.mg_cycles_min <= info.mg_cycles_max <= 3


def test_discrete_solution_is_what_the_errors_measure():
    """The stopped iterate is within 1% of the table's error of the exact
    discrete solution (SuperLU), so Table 3 pins the discretisation."""
    N, eps = 256, 1e-6
    p = problem(N, eps)
    u, f = parabolic_mms(eps, p.x, p.y)
    Ue = spla.splu(p.csr().tocsc()).solve(f)
    err, _ = table_case(N, eps)
    assert np.abs(Ue - u).max() == pytest.approx(err, rel=1e-2)
