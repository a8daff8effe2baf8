"""Pins of the oracle on other layer-adapted meshes (Sec. 2.2's remark on the
general Shishkin mesh with a layer fraction q = nl / N; Sec. 3's statement
that the preconditioner needs only a transition point between layer and
interior; the remark after Thm. big_bound that graded, Bakhvalov-type layer
meshes are covered).

None retypes the mesh formulas: the Bakhvalov-Shishkin layer is pinned by
the equidistribution property that defines it, by the first-order,
eps-uniform convergence that is its purpose (upwind on such meshes is
O(N^-1), against O(N^-1 ln N) on Shishkin meshes), and the general meshes by
the structure of M-hat, exact region solves and dense LU, as on the paper's
mesh."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_2108_13468_amd import inputs
from tests.mms import exponential_mms


def mms_problem(N, eps, kind="shishkin", nl=None):
    inst = inputs.mms_exponential(N, eps)
    return O.Problem(N, eps, c1=inst.c1_at, c2=inst.c2_at, r=1.0, sigma=inst.sigma,
                     clow_x=inst.clow[0], clow_y=inst.clow[1], mesh_kind=kind, layer_cells=nl)


def plain(N, eps, kind="shishkin", nl=None):
    inst = inputs.plain(N, eps)
    return O.Problem(N, eps, c1=inst.c1_at, c2=inst.c2_at, r=1.0, mesh_kind=kind,
                     layer_cells=nl)


def mms_error(N, eps, kind="shishkin", nl=None):
    p = mms_problem(N, eps, kind, nl)
    u, f = exponential_mms(eps, p.x, p.y)
    return np.abs(spla.spsolve(p.csr().tocsc(), f) - u).max()


# ---------------------------------------------------------------- meshes ----

@pytest.mark.parametrize("N,eps,nl", [(64, 1e-4, 32), (256, 1e-6, 64), (512, 1e-8, 384)])
def test_bakhvalov_shishkin_equidistributes_the_layer_function(N, eps, nl):
    """The layer nodes make exp(-clow x / (sigma eps)) fall in equal steps
    from 1 at x = 0 to 1/N at the transition point, which lies at
    sigma eps ln(N) / clow; the interior cells are equal; widths are
    positive, grow through the layer and add up to 1."""
    sigma, clow = 2.5, 2.0
    tau, x, w = O.mesh_axis(N, eps, sigma, clow, "bakhvalov-shishkin", nl)
    s = sigma * eps / clow
    assert tau == pytest.approx(s * np.log(N), rel=1e-15)
    assert x[nl] == tau and x[N] == pytest.approx(1.0, abs=1e-15)
    e = np.exp(-x[: nl + 1] / s)
    steps = np.diff(e)
    np.testing.assert_allclose(steps, -(1 - 1 / N) / nl, rtol=1e-9)
    assert e[nl] == pytest.approx(1.0 / N, rel=1e-12)
    wl = w[1: nl + 1]
    assert np.all(wl > 0) and np.all(np.diff(wl) > 0)
    np.testing.assert_allclose(wl, np.diff(x[: nl + 1]), rtol=1e-9)
    np.testing.assert_allclose(w[nl + 1:], (1 - tau) / (N - nl), rtol=1e-15)
    assert w[1:].sum() == pytest.approx(1.0, abs=1e-14)


def test_general_shishkin_mesh():
    """q = nl/N: nl equal layer cells on [0, min(q, sigma eps ln N / clow)];
    nl = N/2 is the paper's mesh exactly; a large eps gives the uniform mesh
    for either kind."""
    N, eps = 256, 1e-5
    for nl in (64, 192):
        tau, x, w = O.mesh_axis(N, eps, 2.0, 1.0, "shishkin", nl)
        assert tau == pytest.approx(min(nl / N, 2 * eps * np.log(N)), rel=1e-15)
        np.testing.assert_allclose(w[1: nl + 1], tau / nl, rtol=1e-15)
        np.testing.assert_allclose(w[nl + 1:], (1 - tau) / (N - nl), rtol=1e-15)
    t0, x0, w0 = O.mesh_axis(N, eps, 2.0, 1.0)
    t1, x1, w1 = O.mesh_axis(N, eps, 2.0, 1.0, "shishkin", N // 2)
    assert t0 == t1 and np.array_equal(x0, x1) and np.array_equal(w0, w1)
    for kind in ("shishkin", "bakhvalov-shishkin"):
        _, x, _ = O.mesh_axis(N, 0.5, 2.0, 1.0, kind, 64)
        np.testing.assert_allclose(x, np.arange(N + 1) / N, rtol=1e-14, atol=1e-16)


# ------------------------------------------------------- discretisation ----

def test_bakhvalov_shishkin_first_order_uniformly_in_eps():
    """Upwind differences on a Bakhvalov-Shishkin mesh converge at first order
    in N, uniformly in eps, without the ln N factor of the Shishkin mesh:
    on the paper's exponential manufactured solution the observed rates
    rise towards 1 (above 0.93 from N = 64), the errors do not depend on eps,
    and they are below the Shishkin errors at every N."""
    errs = {eps: [mms_error(N, eps, "bakhvalov-shishkin") for N in (64, 128, 256)]
            for eps in (1e-4, 1e-8)}
    for eps, e in errs.items():
        rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(rates > 0.93) and rates[1] > rates[0], (eps, rates)
    np.testing.assert_allclose(errs[1e-4], errs[1e-8], rtol=5e-3)
    shi = [mms_error(N, 1e-8) for N in (64, 128, 256)]
    assert np.all(np.array(errs[1e-8]) < 0.6 * np.array(shi))


def test_general_shishkin_almost_first_order():
    """With a quarter of the cells in the layer the Shishkin error keeps its
    N^-1 ln N behaviour: rates below 1 and rising, errors independent of
    eps."""
    e6 = [mms_error(N, 1e-6, nl=N // 4) for N in (64, 128, 256)]
    e8 = [mms_error(N, 1e-8, nl=N // 4) for N in (64, 128, 256)]
    rates = np.log2(np.array(e6[:-1]) / np.array(e6[1:]))
    assert np.all((0.5 < rates) & (rates < 0.85)) and rates[1] > rates[0]
    np.testing.assert_allclose(e6, e8, rtol=5e-3)


# ------------------------------------------------------- preconditioner ----

def extract(op, n):
    return np.column_stack([op(e) for e in np.eye(n)])


@pytest.mark.parametrize("kind,N,nl", [("shishkin", 16, 4), ("shishkin", 16, 12),
                                       ("bakhvalov-shishkin", 16, 8),
                                       ("bakhvalov-shishkin", 20, 6)])
def test_mhat_structure_general_meshes(kind, N, nl):
    """M-hat = A with the West entries dropped on rows i > nl and the South
    entries on rows j > nl (the regions of Sec. 3.1 follow the transition
    point), as on the paper's mesh."""
    p = plain(N, 1e-5, kind, nl)
    A = p.csr().toarray()
    M = np.linalg.inv(extract(lambda b: p.M_inv(b, corner="exact"), p.n))
    Nh = M - A
    scale = np.abs(A).max()
    Nh[np.abs(Nh) < 1e-9 * scale] = 0.0
    n1 = N - 1
    expect = np.zeros_like(A)
    for j in range(1, N):
        for i in range(1, N):
            pr = (j - 1) * n1 + (i - 1)
            if i > nl and i > 1:
                expect[pr, pr - 1] = -A[pr, pr - 1]
            if j > nl and j > 1:
                expect[pr, pr - n1] = -A[pr, pr - n1]
    np.testing.assert_allclose(Nh, expect, rtol=1e-7, atol=1e-9 * scale)
    assert np.all(Nh >= 0)


@pytest.mark.parametrize("kind,nl", [("shishkin", 8), ("bakhvalov-shishkin", 16)])
def test_fgmres_and_corner_mg_on_general_meshes(kind, nl):
    """FGMRES with M reaches the dense-LU solution; the corner cycle, run to
    convergence, reaches the exact corner solve."""
    N = 32
    p = plain(N, 1e-4, kind, nl)
    A = p.csr().toarray()
    F = np.random.default_rng(5).standard_normal(p.n)
    u, st, _, _ = p.fgmres(F, tol=1e-12, scaled=True, mg_maxcyc=200)
    assert st == 0
    ue = np.linalg.solve(A, F)
    assert np.abs(u - ue).max() <= 1e-9 * np.abs(ue).max()
    bC = np.random.default_rng(6).standard_normal(nl * nl)
    z, cyc = p.corner_mg(bC, rtol=1e-13, maxcyc=2000)
    ze = p.corner_exact(bC)
    assert np.abs(z - ze).max() <= 1e-10 * np.abs(ze).max()


def test_mhat_iterations_do_not_depend_on_the_layer_mesh():
    """With the exact corner solve (M-hat), FGMRES needs the same number of
    iterations on the Bakhvalov-Shishkin mesh as on the Shishkin mesh: the
    preconditioner's bound holds for any layer mesh (remark after Thm.
    big_bound)."""
    for N, eps in ((64, 1e-4), (128, 1e-6)):
        its = []
        for kind in ("shishkin", "bakhvalov-shishkin"):
            inst = inputs.plain(N, eps, seed=1)
            p = plain(N, eps, kind)
            F = O.sine_series(N, p.x, p.y, inst.a)
            _, st, info, _ = p.fgmres(F, tol=1e-8, scaled=True, corner="exact")
            assert st == 0
            its.append(info.iterations)
        assert abs(its[0] - its[1]) <= 1, (N, eps, its)
