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
