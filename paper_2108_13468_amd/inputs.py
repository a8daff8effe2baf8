"""Seeded synthetic inputs for the workloads (problem data only).

This module draws random numbers and describes problem instances; it holds
none of the method's arithmetic (no mesh, stencil, solver or projection).
Both the CPU oracle side (tests) and the GPU side (tests, smoke, bench) take
their inputs from here, so the two see identical data.

Instances follow the model problem  -eps Lap u - c . grad u + r u = f  on the
unit square with zero Dirichlet data (Sec. 1, eq. 2D; Sec. 3):
  * c1(x) = c1[0] + c1[1] x + c1[2] x^2 and c2(y) likewise (polynomials in
    one variable each);
  * r is a constant, or bilinear on an m x m uniform control grid
    (controls stored x-fastest, R[q*m + p]);
  * f is a tensor sine series  sum_{k,l} a[l-1, k-1] sin(k pi x) sin(l pi y).
Random draws use numpy's PCG64 (numpy.random.default_rng).
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


@dataclass
class Instance:
    N: int
    eps: float
    c1: Tuple[float, float, float] = (1.0, 0.0, 1.0)   # 1 + x^2
    c2: Tuple[float, float, float] = (1.0, 1.0, 0.0)   # 1 + y
    r_const: Optional[float] = 1.0
    r_ctrl: Optional[np.ndarray] = None                 # m x m, [q, p]
    a: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))  # [l-1, k-1]
    sigma: float = 2.0
    clow: Tuple[float, float] = (1.0, 1.0)
    mesh_kind: str = "shishkin"          # or "bakhvalov-shishkin"
    layer_cells: Optional[int] = None    # cells on [0, tau] per axis (None: N/2)
    y_layer: str = "exponential"         # or "parabolic" (c2 = 0: layer width sqrt(eps))

    def c1_at(self, x):
        c = self.c1
        return c[0] + c[1] * np.asarray(x) + c[2] * np.asarray(x) ** 2

    def c2_at(self, y):
        c = self.c2
        return c[0] + c[1] * np.asarray(y) + c[2] * np.asarray(y) ** 2


def plain(N, eps, seed=0, K=3):
    """N x N mesh, c = (1+x^2, 1+y), r = 1, 3x3 sine series with a ~ U(-1,1),
    Shishkin transition tau = min(1/2, 2 eps ln N)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(K, K))
    return Instance(N=N, eps=eps, a=a)


def small_case(seed=0):
    """N = 64, eps = 1e-2 (63^2 unknowns)."""
    return plain(64, 1e-2, seed)


def headline_case(eps=1e-6, seed=1):
    """N = 1024, eps in {1e-2, 1e-4, 1e-6} (1023^2 unknowns)."""
    return plain(1024, eps, seed)


def batch_cases(count=64, seed=2, sizes=(128, 256, 512, 1024)):
    """Uneven batch: N ~ U{sizes} (the workload: {128,256,512,1024}),
    log10 eps ~ U(-8,-2), c = (1 + a x, 1 + b y) with a, b ~ U(0,1),
    r ~ U(0.5, 2) constant, 3x3 sine series with a_kl ~ U(-1,1).  Per
    instance the draw order is a_kl (row-major), r, a, b, N, eps."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        akl = rng.uniform(-1.0, 1.0, size=(3, 3))
        r = rng.uniform(0.5, 2.0)
        ca = rng.uniform(0.0, 1.0)
        cb = rng.uniform(0.0, 1.0)
        N = int(rng.choice(list(sizes)))
        eps = float(10.0 ** rng.uniform(-8.0, -2.0))
        out.append(Instance(N=N, eps=eps, c1=(1.0, ca, 0.0), c2=(1.0, cb, 0.0),
                            r_const=r, a=akl))
    return out


@dataclass
class AdjointCase:
    inst: Instance            # the parameter set the gradient is taken at
    a_ref: np.ndarray         # reference sine coefficients (16 x 16)
    R_ref: np.ndarray         # reference bilinear controls (4 x 4)
    noise: np.ndarray         # N(0, sd) per interior node, added to u_ref


def adjoint_case(N=512, eps=1e-4, K=16, m=4, noise_sd=1e-3, seed=3):
    """Misfit J = 0.5 ||u - u_obs||^2 with u_obs = u(a_ref, R_ref) + noise.
    a ~ U(-1,1) (K x K), bilinear r controls ~ U(0.5, 2) (m x m); the
    gradient is evaluated at a second draw (a, R).  Draw order: a_ref, R_ref,
    a, R, noise."""
    rng = np.random.default_rng(seed)
    a_ref = rng.uniform(-1.0, 1.0, size=(K, K))
    R_ref = rng.uniform(0.5, 2.0, size=(m, m))
    a = rng.uniform(-1.0, 1.0, size=(K, K))
    R = rng.uniform(0.5, 2.0, size=(m, m))
    noise = rng.normal(0.0, noise_sd, size=(N - 1) ** 2)
    inst = Instance(N=N, eps=eps, r_const=None, r_ctrl=R, a=a)
    return AdjointCase(inst=inst, a_ref=a_ref, R_ref=R_ref, noise=noise)


def multi_rhs_case(N=2048, eps=1e-6, nrhs=16, seed=4):
    """N = 2048, eps = 1e-6, nrhs seeded 3x3 sine series sharing one operator
    (c = (1+x^2, 1+y), r = 1)."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1.0, 1.0, size=(nrhs, 3, 3))
    return Instance(N=N, eps=eps), A


def mms_exponential(N, eps):
    """The paper's two-exponential-layer test (Sec. 3.3): c = (2, 3), r = 1,
    sigma = 5/2, lower bounds (2, 3); f is supplied by the manufactured
    solution (see tests)."""
    return Instance(N=N, eps=eps, c1=(2.0, 0.0, 0.0), c2=(3.0, 0.0, 0.0),
                    r_const=1.0, sigma=2.5, clow=(2.0, 3.0))


def mms_parabolic(N, eps):
    """The paper's test with one parabolic and one exponential layer (Sec.
    3.3): -eps Lap u - u_x + u = f, so c = (1, 0), r = 1; sigma = 5/2; the
    x-layer mesh takes the lower bound Clow = 0.99 of c1 = 1 (the bound the
    one-dimensional tables are reproduced with); the y-axis transition point
    is sigma sqrt(eps) ln N.  f is supplied by the manufactured solution (see
    tests)."""
    return Instance(N=N, eps=eps, c1=(1.0, 0.0, 0.0), c2=(0.0, 0.0, 0.0), r_const=1.0,
                    sigma=2.5, clow=(0.99, 1.0), y_layer="parabolic")
