"""Dense brute force of H_a on tiny grids (TEST INFRASTRUCTURE).

Every operator is an explicit matrix: the 2-D DFT is built from the DFT
definition (no FFT library), the staggered gradients and fractional
Laplacians are F^-1 diag(symbol) F, and the one-step map is assembled from
the paper's block form of T (eq Tprod) with the blocks D, E, G of eqs D4, E,
G4 and the source map of eqs s2, s3.  H_a is then the recursion of
Definition 4 written with these matrices.  This is a different route to the
same operator than `kspace.forward`, so the two check each other.

Symbols and diagonals are taken from `kspace.Operators` (its symbol tables are
pinned separately by the closed-form tests); only the time stepping and the
adjoint are re-derived here.
"""
from __future__ import annotations

import numpy as np

from .kspace import D, Operators


def dft_matrix(n: int) -> np.ndarray:
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


class DenseModel:
    def __init__(self, prm: dict, c0, rho0):
        op = Operators(prm, c0, rho0)
        nx, ny = prm["nx"], prm["ny"]
        N = nx * ny
        self.N, self.op, self.prm = N, op, prm
        dt = prm["dt"]
        # 2-D DFT for row-major [ny, nx] flattening: kron(F_y, F_x)
        F = np.kron(dft_matrix(ny), dft_matrix(nx))
        Fi = np.conj(F) / N

        def spec(m):
            M = Fi @ (m.reshape(-1)[:, None] * F)
            assert np.abs(M.imag).max() < 1e-9 * max(1.0, np.abs(M.real).max())
            return M.real

        I = np.eye(N)
        Z = np.zeros((N, N))
        diag = lambda a: np.diag(np.broadcast_to(a, (ny, nx)).reshape(-1))
        self.Gxp, self.Gyp = spec(op.mxp), spec(op.myp)
        self.Gxm, self.Gym = spec(op.mxm), spec(op.mym)
        Ydis, Yabs = spec(op.ldis), spec(op.labs)
        C = diag(op.c2)
        eta, tau = diag(op.eta), diag(op.tau)
        # stacked (d = 2) diagonal blocks
        blk = lambda a, b: np.block([[a, Z], [Z, b]])
        Q = blk(diag(op.rho0), diag(op.rho0))
        Qs_inv = blk(diag(1.0 / op.rhox), diag(1.0 / op.rhoy))
        Av = blk(diag(op.avx), diag(op.avy))
        Ar = blk(diag(op.arx), diag(op.ary))
        Phi = -dt * blk(self.Gxp, self.Gyp)     # eq phi
        Psi = -dt * blk(self.Gxm, self.Gym)     # eq psi
        one = np.vstack([I, I])                  # 1_i (x) : R^N -> R^{dN}
        Sig = np.hstack([I, I])                  # sum_i  : R^{dN} -> R^N
        Pdis = C @ (I - eta @ Ydis)
        Pfull = C @ (I - eta @ Ydis - tau @ Yabs / dt)
        Dm = Pfull @ Sig @ (Ar @ Q @ Psi @ Av @ Av)                       # eq D4
        Em = Pdis @ Sig @ (Ar @ Ar)                                      # eq E
        Gm = Pfull @ Sig @ (Ar @ Q @ Psi @ Av @ Qs_inv @ Phi @ one)      # eq G4
        Zd = np.zeros((2 * N, 2 * N))
        T = np.block([
            [Av @ Av, Zd, Av @ Qs_inv @ Phi @ one],
            [Ar @ Q @ Psi @ Av @ Av, Ar @ Ar, Ar @ Q @ Psi @ Av @ Qs_inv @ Phi @ one],
            [Dm, Em, Gm],
        ])                                                               # eq Tprod
        self.T = T
        Isz = np.vstack([np.zeros((2 * N, 2 * N)), np.eye(2 * N), Pdis @ Sig])   # eq s3
        self.Src = Isz @ one @ diag(1.0 / (2.0 * D * op.c2))             # eq s2 (S = I)
        Mrow = np.zeros((len(op.tap_w), N))
        for s in range(len(op.tap_w)):
            for t in range(4):
                Mrow[s, op.tap_idx[s, t]] += op.tap_w[s, t]
        self.M = Mrow
        self.Mz = np.hstack([np.zeros((len(op.tap_w), 4 * N)), Mrow])   # M I_z^p

    def H(self) -> np.ndarray:
        """Dense H_a of Definition 4: [nt*ns, N], time-major rows."""
        nt = self.prm["nt"]
        ns = self.M.shape[0]
        Zs = np.zeros((5 * self.N, self.N))      # z_{-1} = 0, one column per unit p0
        H = np.zeros((nt, ns, self.N))
        for n in range(-1, nt - 1):
            Zs = self.T @ Zs + (self.Src if n in (-1, 0) else 0.0)
            H[n + 1] = self.Mz @ Zs
        return H.reshape(nt * ns, self.N)
