"""Shared helpers of the GPU parity tests (imported only by tests)."""
import numpy as np

from lattice_inputs import gauge_field


def torch_dev():
    import torch
    return torch.device("cuda:0")


def to_gpu(x_np):
    """numpy (nrhs, sites, dof) complex -> torch dof-major (dof, sites, nrhs)."""
    import torch
    from paper_2509_11424_amd import to_dofmajor
    return torch.from_numpy(to_dofmajor(x_np)).to(torch_dev())


def from_gpu(t):
    from paper_2509_11424_amd import from_dofmajor
    return from_dofmajor(t.cpu().numpy())


def flat_to_sites(v, dof):
    """oracle flat vectors [..., n] -> [..., sites, dof]"""
    return v.reshape(v.shape[:-1] + (-1, dof))


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class Setup:
    """A lattice, its oracle operator and (lazily) the GPU objects."""

    def __init__(self, dims, eps, seed, m0, csw):
        from oracle.dirac import WilsonClover
        self.dims = dims
        self.U = gauge_field(dims, eps, seed)
        self.m0, self.csw = m0, csw
        self.D = WilsonClover(self.U, m0, csw)
        self.V = self.D.V


class LocalStencil:
    """Evaluates (D x)(s) at one site from the oracle's building blocks."""

    def __init__(self, U, m0, csw):
        from oracle import dirac
        self.U, self.m0, self.csw = U, m0, csw
        self.dirac = dirac
        self.T, self.Z, self.Y, self.X = U.shape[:4]

    def _idx(self, c):
        x, y, z, t = c
        return x % self.X + self.X * (y % self.Y + self.Y * (z % self.Z + self.Z * (t % self.T)))

    def at(self, s, x):
        d = self.dirac
        X, Y, Z, T = self.X, self.Y, self.Z, self.T
        c = [s % X, (s // X) % Y, (s // (X * Y)) % Z, s // (X * Y * Z)]
        # clover from a 3^4 patch around the site (periodic copy of the field)
        patch = np.zeros((3, 3, 3, 3, 4, 3, 3), dtype=complex)
        for dt in range(3):
            for dz in range(3):
                for dy in range(3):
                    for dx in range(3):
                        cc = (c[0] + dx - 1, c[1] + dy - 1, c[2] + dz - 1, c[3] + dt - 1)
                        patch[dt, dz, dy, dx] = self.U[cc[3] % T, cc[2] % Z, cc[1] % Y, cc[0] % X]
        Cl = d.clover_matrix(patch, self.csw)[1, 1, 1, 1]
        out = (4 + self.m0) * x[s] + Cl @ x[s]
        g = d.gammas()
        I4 = np.eye(4)
        for mu in range(4):
            e = [0, 0, 0, 0]
            e[mu] = 1
            cf = [c[i] + e[i] for i in range(4)]
            cb = [c[i] - e[i] for i in range(4)]
            ph_f = -1.0 if (mu == 3 and c[3] == T - 1) else 1.0
            ph_b = -1.0 if (mu == 3 and c[3] == 0) else 1.0
            Uf = self.U[c[3], c[2], c[1], c[0], mu]
            Ub = self.U[cb[3] % T, cb[2] % Z, cb[1] % Y, cb[0] % X, mu].conj().T
            pf = x[self._idx(cf)].reshape(4, 3)
            pb = x[self._idx(cb)].reshape(4, 3)
            out = out - 0.5 * ph_f * ((I4 - g[mu]) @ (pf @ Uf.T)).reshape(12)
            out = out - 0.5 * ph_b * ((I4 + g[mu]) @ (pb @ Ub.T)).reshape(12)
        return out
