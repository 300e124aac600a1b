"""Oracle of the optical operators of Section 3.1: the diffusion approximation
with the Robin boundary condition (eq DA) discretised by first-order Galerkin
FEM (eqs var_fo, var_fr, var_f_adj, system_forward2), the heating map
H = mu o I Phi (eq forward_out), its matrix-free Frechet derivative J_o
(eq dh_des) and the adjoint J_o^* (eqs system_adjoint, system_adjoint1,
prodtproj), in 2-D.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never imports it.

Readings (the paper's meshes are not available):
  * Mesh matched to the acoustic grid: every acoustic node (j, i) is the
    centre of a square pixel of side dx (Section 6.1: two elements form a
    pixel whose centre is an acoustic node).  FEM nodes are the pixel
    corners, (ny + 1) x (nx + 1) of them, numbered row-major; pixel (j, i)
    is split along its diagonal from corner (j, i) to corner (j + 1, i + 1)
    into element 2 (j nx + i) (corners (j,i), (j,i+1), (j+1,i+1)) and
    element 2 (j nx + i) + 1 (corners (j,i), (j+1,i+1), (j+1,i)).
  * Illumination q is a constant inward current I_s on a set of the four
    sides ("left", "right", "bottom", "top"); gamma_2 = 1/pi.
  * The initial pressure at an acoustic node is the mean of the heating of
    its pixel's two elements (the L2 projection onto pixel constants; both
    elements have the same area), with Gruneisen Gamma = 1.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GAMMA_2 = 1.0 / math.pi


class Mesh:
    """Grid-matched P1 triangulation of nx x ny pixels of side dx."""

    def __init__(self, nx: int, ny: int, dx: float):
        self.nx, self.ny, self.dx = nx, ny, dx
        self.nn = (nx + 1) * (ny + 1)
        self.ne = 2 * nx * ny
        node = lambda j, i: j * (nx + 1) + i
        tri = np.zeros((self.ne, 3), dtype=np.int64)
        for j in range(ny):
            for i in range(nx):
                e = 2 * (j * nx + i)
                tri[e] = (node(j, i), node(j, i + 1), node(j + 1, i + 1))
                tri[e + 1] = (node(j, i), node(j + 1, i + 1), node(j + 1, i))
        self.tri = tri
        jj, ii = np.divmod(np.arange(self.nn), nx + 1)
        # node coordinates: pixel (j, i) is centred on acoustic node ((i - nx/2) dx, (j - ny/2) dx)
        self.xy = np.stack([(ii - nx / 2 - 0.5) * dx, (jj - ny / 2 - 0.5) * dx], axis=1)
        self.area = np.full(self.ne, 0.5 * dx * dx)
        # gradients of the three hat functions on every element: [ne, 3, 2]
        g = np.zeros((self.ne, 3, 2))
        for e in range(self.ne):
            P = self.xy[tri[e]]
            M = np.array([[1.0, P[0, 0], P[0, 1]], [1.0, P[1, 0], P[1, 1]], [1.0, P[2, 0], P[2, 1]]])
            coef = np.linalg.inv(M)          # columns: coefficients (a, b, c) of each hat a + b x + c y
            g[e] = coef[1:, :].T
        self.grad = g
        # boundary edges per side: list of node pairs
        self.sides = {
            "bottom": [(node(0, i), node(0, i + 1)) for i in range(nx)],
            "top": [(node(ny, i), node(ny, i + 1)) for i in range(nx)],
            "left": [(node(j, 0), node(j + 1, 0)) for j in range(ny)],
            "right": [(node(j, nx), node(j + 1, nx)) for j in range(ny)],
        }

    def boundary_edges(self):
        return [e for s in ("bottom", "top", "left", "right") for e in self.sides[s]]


def stiffness(mesh: Mesh, kappa_e: np.ndarray) -> sp.csr_matrix:
    """K[kappa]_kp = sum over elements of kappa_e * S_e * grad phi_k . grad phi_p."""
    rows, cols, vals = [], [], []
    for e in range(mesh.ne):
        Ke = kappa_e[e] * mesh.area[e] * mesh.grad[e] @ mesh.grad[e].T
        for a in range(3):
            for b in range(3):
                rows.append(mesh.tri[e, a]); cols.append(mesh.tri[e, b]); vals.append(Ke[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.nn, mesh.nn))


def mass(mesh: Mesh, mu_e: np.ndarray) -> sp.csr_matrix:
    """C[mu]_kp = sum over elements of mu_e * int phi_k phi_p (P1: S/12 [[2,1,1],[1,2,1],[1,1,2]])."""
    loc = (np.ones((3, 3)) + np.eye(3)) / 12.0
    rows, cols, vals = [], [], []
    for e in range(mesh.ne):
        Ce = mu_e[e] * mesh.area[e] * loc
        for a in range(3):
            for b in range(3):
                rows.append(mesh.tri[e, a]); cols.append(mesh.tri[e, b]); vals.append(Ce[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.nn, mesh.nn))


def robin(mesh: Mesh, gamma: float = GAMMA_2) -> sp.csr_matrix:
    """R_kp = 2 gamma int_boundary phi_k phi_p ds (edge P1 mass L/6 [[2,1],[1,2]])."""
    rows, cols, vals = [], [], []
    for (a, b) in mesh.boundary_edges():
        L = np.linalg.norm(mesh.xy[a] - mesh.xy[b])
        for (p, q, w) in ((a, a, 2), (b, b, 2), (a, b, 1), (b, a, 1)):
            rows.append(p); cols.append(q); vals.append(2.0 * gamma * L * w / 6.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.nn, mesh.nn))


NORMALS = {"bottom": (0.0, -1.0), "top": (0.0, 1.0), "left": (-1.0, 0.0), "right": (1.0, 0.0)}


def load(mesh: Mesh, sides, current: float = 1.0, func=None) -> np.ndarray:
    """G_p = int_boundary 2 I_s phi_p ds for a constant current on `sides`
    (or, with `func(x, y, normal)`, a current given pointwise on every side,
    integrated by the exact P1 rule for its linear interpolant on each edge)."""
    G = np.zeros(mesh.nn)
    for side, edges in mesh.sides.items():
        if func is None and side not in sides:
            continue
        for (a, b) in edges:
            L = np.linalg.norm(mesh.xy[a] - mesh.xy[b])
            if func is None:
                G[a] += 2.0 * current * L / 2.0
                G[b] += 2.0 * current * L / 2.0
            else:
                fa, fb = func(*mesh.xy[a], NORMALS[side]), func(*mesh.xy[b], NORMALS[side])
                G[a] += 2.0 * L * (2 * fa + fb) / 6.0
                G[b] += 2.0 * L * (fa + 2 * fb) / 6.0
    return G


def system(mesh: Mesh, kappa_e, mu_e, gamma: float = GAMMA_2) -> sp.csr_matrix:
    """A_o = K[kappa] + C[mu] + R (eq system_forward2)."""
    return (stiffness(mesh, kappa_e) + mass(mesh, mu_e) + robin(mesh, gamma)).tocsr()


def node_to_element(mesh: Mesh, theta: np.ndarray) -> np.ndarray:
    """(I theta)_j = mean of theta over the three nodes of element j (eq intp1)."""
    return theta[mesh.tri].mean(axis=1)


def element_to_node(mesh: Mesh, Theta: np.ndarray) -> np.ndarray:
    """(I^+ Theta)_p = (1/3) sum over elements j at p of S_j Theta_j (eq intp)."""
    out = np.zeros(mesh.nn)
    np.add.at(out, mesh.tri.reshape(-1), np.repeat(mesh.area * Theta / 3.0, 3))
    return out


def forward(mesh: Mesh, kappa_e, mu_e, G: np.ndarray):
    """H_o: Phi solves A_o Phi = G (eq system_forward), H = mu o I Phi
    (eq forward_out).  Returns (H, Phi)."""
    A = system(mesh, kappa_e, mu_e)
    Phi = spla.spsolve(A.tocsc(), G)
    return np.asarray(mu_e) * node_to_element(mesh, Phi), Phi


def jacobian(mesh: Mesh, kappa_e, mu_e, Phi0, dkappa, dmu) -> np.ndarray:
    """J_o [dkappa, dmu] (eq dh_des): A_o dPhi = -(K[dkappa] + C[dmu]) Phi0,
    dH = dmu o I Phi0 + mu o I dPhi."""
    A = system(mesh, kappa_e, mu_e)
    rhs = -(stiffness(mesh, dkappa) + mass(mesh, dmu)) @ Phi0
    dPhi = spla.spsolve(A.tocsc(), rhs)
    return np.asarray(dmu) * node_to_element(mesh, Phi0) + np.asarray(mu_e) * node_to_element(mesh, dPhi)


def jacobian_adjoint(mesh: Mesh, kappa_e, mu_e, Phi0, H) -> tuple[np.ndarray, np.ndarray]:
    """J_o^* H by adjoint-then-discretise (eqs system_adjoint, system_adjoint1,
    prodtproj): A_o Htil = -I^+(mu o H); per element j the kappa part is
    grad Htil . grad Phi0 and the mu part is (1/S_j) Htil^T (dA/dmu_j) Phi0 +
    H_j (I Phi0)_j."""
    A = system(mesh, kappa_e, mu_e)
    Ht = spla.spsolve(A.tocsc(), -element_to_node(mesh, np.asarray(mu_e) * H))
    gH = np.einsum("eab,ea->eb", mesh.grad, Ht[mesh.tri])
    gP = np.einsum("eab,ea->eb", mesh.grad, Phi0[mesh.tri])
    dk = np.sum(gH * gP, axis=1)
    loc = (np.ones((3, 3)) + np.eye(3)) / 12.0
    dm = np.einsum("ea,ab,eb->e", Ht[mesh.tri], loc, Phi0[mesh.tri]) + H * node_to_element(mesh, Phi0)
    return dk, dm


def jacobian_adjoint_discrete(mesh: Mesh, kappa_e, mu_e, Phi0, H) -> tuple[np.ndarray, np.ndarray]:
    """The discretise-then-adjoint form (eq num_adj): the Euclidean transpose
    of `jacobian`, by dense assembly of dA/dkappa_j and dA/dmu_j (tiny meshes)."""
    A = system(mesh, kappa_e, mu_e).toarray()
    ne = mesh.ne
    Ii = np.zeros((ne, mesh.nn))
    for j in range(ne):
        Ii[j, mesh.tri[j]] = 1.0 / 3.0
    w = np.linalg.solve(A.T, Ii.T @ (np.asarray(mu_e) * H))   # (I A^-1)^T (mu o H)
    dk = np.zeros(ne)
    dm = np.zeros(ne)
    for j in range(ne):
        ej = np.zeros(ne); ej[j] = 1.0
        dk[j] = w @ (-(stiffness(mesh, ej) @ Phi0))
        dm[j] = w @ (-(mass(mesh, ej) @ Phi0))
    return dk, dm + H * (Ii @ Phi0)


def pixel_mean(mesh: Mesh, H: np.ndarray) -> np.ndarray:
    """Initial pressure on the acoustic grid: the mean of each pixel's two
    elements, [ny][nx] (Gruneisen 1)."""
    return H.reshape(mesh.ny, mesh.nx, 2).mean(axis=2)


def pixel_mean_T(mesh: Mesh, p: np.ndarray) -> np.ndarray:
    """Transpose of pixel_mean: half of each pixel value to each of its elements."""
    return np.repeat(0.5 * np.asarray(p).reshape(-1), 2)
