"""Pins of the optical oracle (oracle/optical.py) against what the paper and
the mathematics fix: FEM assembly identities, an exact solution of the
diffusion approximation with its Robin condition reached at second order,
J_o against finite differences of H_o, J_o^* as the adjoint of J_o, and the
equality of the adjoint-then-discretise and discretise-then-adjoint forms on
the equal-area mesh (the paper's remark after eq prodtproj)."""
import math

import numpy as np
import pytest

import qpat_inputs as qi
from oracle import optical as O


def coeffs(mesh, seed):
    """Tissue-like optical coefficients per element (mm^-1 scaled to m^-1):
    mu around 0.01 /mm, kappa = 1 / (3 (mu + mu_s')) with mu_s' around 1 /mm."""
    rng = np.random.default_rng(seed)
    mu = 10.0 * (1.0 + 0.5 * rng.uniform(size=mesh.ne))
    mus = 1000.0 * (1.0 + 0.3 * rng.uniform(size=mesh.ne))
    return 1.0 / (3.0 * (mu + mus)), mu


def test_assembly_identities():
    m = O.Mesh(6, 5, 1e-4)
    kap, mu = coeffs(m, 1)
    K, C, R = O.stiffness(m, kap), O.mass(m, mu), O.robin(m)
    one = np.ones(m.nn)
    assert np.abs(K @ one).max() <= 1e-12 * np.abs(K).max()           # constants are in the kernel of K
    assert abs(one @ C @ one - np.sum(mu * m.area)) <= 1e-12 * np.sum(mu * m.area)
    per = 2 * (6 + 5) * 1e-4
    assert abs(one @ R @ one - 2 * O.GAMMA_2 * per) <= 1e-12 * per
    for M in (K, C, R):
        assert abs(M - M.T).max() <= 1e-15 * abs(M).max()
    assert np.all(np.linalg.eigvalsh(O.system(m, kap, mu).toarray()) > 0)
    assert m.area.sum() == pytest.approx(6 * 5 * 1e-8, rel=1e-12)


def test_exact_solution_second_order():
    """phi = exp(a x + b y) with kappa (a^2 + b^2) = mu solves
    -div(kappa grad phi) + mu phi = 0; its Robin data
    I = gamma phi + (kappa/2) d phi/dn drive the FEM solve, and the nodal error
    falls by about 4 when the mesh is refined by 2."""
    kap, mu = 3e-4, 12.0
    a, b = 120.0, 150.0
    s = math.sqrt(mu / kap) / math.hypot(a, b)
    a, b = a * s, b * s
    phi = lambda x, y: math.exp(a * x + b * y)
    errs = []
    for n, dx in ((16, 1e-4), (32, 0.5e-4)):
        m = O.Mesh(n, n, dx)

        def current(x, y, nrm):
            dn = a * nrm[0] + b * nrm[1]
            return O.GAMMA_2 * phi(x, y) + 0.5 * kap * dn * phi(x, y)

        G = O.load(m, None, func=current)
        A = O.system(m, np.full(m.ne, kap), np.full(m.ne, mu))
        Phi = np.linalg.solve(A.toarray(), G)
        ex = np.array([phi(x, y) for x, y in m.xy])
        errs.append(np.abs(Phi - ex).max() / np.abs(ex).max())
    assert errs[1] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_jacobian_matches_finite_differences():
    m = O.Mesh(8, 7, 1e-4)
    kap, mu = coeffs(m, 2)
    G = O.load(m, ["left", "bottom"])
    H0, Phi0 = O.forward(m, kap, mu, G)
    rng = np.random.default_rng(3)
    dk = kap * rng.standard_normal(m.ne)
    dm = mu * rng.standard_normal(m.ne)
    J = O.jacobian(m, kap, mu, Phi0, dk, dm)
    h = 1e-6
    fd = (O.forward(m, kap + h * dk, mu + h * dm, G)[0] - O.forward(m, kap - h * dk, mu - h * dm, G)[0]) / (2 * h)
    assert np.linalg.norm(fd - J) <= 1e-7 * np.linalg.norm(J)


def test_adjoint_of_jacobian():
    m = O.Mesh(7, 6, 1e-4)
    kap, mu = coeffs(m, 4)
    G = O.load(m, ["top"])
    _, Phi0 = O.forward(m, kap, mu, G)
    rng = np.random.default_rng(5)
    dk, dm, H = (rng.standard_normal(m.ne) for _ in range(3))
    J = O.jacobian(m, kap, mu, Phi0, dk, dm)
    ak, am = O.jacobian_adjoint(m, kap, mu, Phi0, H)
    lhs = np.dot(J, H)
    rhs = np.dot(dk, ak) + np.dot(dm, am)
    assert abs(lhs - rhs) <= 1e-12 * (np.linalg.norm(J) * np.linalg.norm(H) + abs(lhs))


def test_adjoint_forms_agree_on_equal_areas():
    m = O.Mesh(5, 4, 1e-4)
    kap, mu = coeffs(m, 6)
    G = O.load(m, ["left"])
    _, Phi0 = O.forward(m, kap, mu, G)
    H = np.random.default_rng(7).standard_normal(m.ne)
    a = O.jacobian_adjoint(m, kap, mu, Phi0, H)
    b = O.jacobian_adjoint_discrete(m, kap, mu, Phi0, H)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-10 * np.abs(y).max()


def test_pixel_map_and_transpose():
    m = O.Mesh(4, 3, 1e-4)
    H = np.random.default_rng(8).standard_normal(m.ne)
    p = np.random.default_rng(9).standard_normal((3, 4))
    assert np.dot(O.pixel_mean(m, H).ravel(), p.ravel()) == pytest.approx(np.dot(H, O.pixel_mean_T(m, p)), rel=1e-13)
    assert np.allclose(O.pixel_mean(m, np.ones(m.ne)), 1.0)
