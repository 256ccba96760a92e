"""Shared test fixtures: seeded problems and their oracle references."""

import os

import numpy as np
import pytest

import workloads as W
from oracle import assemble, fem, multigrid, solve

MAT = dict(E0=1.0, Emin=1e-9, penal=3.0)


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def need_gpu():
    from paper_2311_05595_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libmgcg.so is not built: the GPU tests need the HIP library")
    if not gpu_available():
        pytest.skip("no GPU")


class Case:
    """A seeded problem with its oracle operator hierarchy."""

    def __init__(self, kind, nel, order=1, nsub=1, nlevels=2, nrhs=1, field="grf", seed=0,
                 precision="fp64", omega=0.6, corr=3.0):
        self.kind, self.nel, self.order, self.nsub = kind, tuple(nel), order, nsub
        self.nlevels, self.nrhs, self.precision, self.omega = nlevels, nrhs, precision, omega
        self.mask, self.f = W.make_problem(kind, *nel, order, nrhs)
        shape = (nel[2] * nsub, nel[1] * nsub, nel[0] * nsub)
        if field == "grf":
            self.rho = W.gaussian_random_field(shape, seed, corr=corr)
        else:
            self.rho = W.uniform_field(shape, seed, 0.05, 1.0)
        self.Ks = fem.sub_element_matrices(order, nsub)
        self._K = None
        self._H = None

    @property
    def dims(self):
        return assemble.node_dims(self.nel, self.order)

    @property
    def K(self):
        if self._K is None:
            self._K = assemble.stiffness(self.rho, self.nel, self.order, self.nsub, self.Ks, **MAT)
        return self._K

    @property
    def H(self):
        if self._H is None:
            A0 = assemble.level_operator(self.K, self.mask)
            self._H = multigrid.Hierarchy(A0, self.mask, self.dims, self.nlevels, order0=self.order)
        return self._H

    def problem(self, **kw):
        from paper_2311_05595_amd import api
        args = dict(order=self.order, nsub=self.nsub, nlevels=self.nlevels,
                    precision=self.precision, omega=self.omega)
        args.update(kw)
        p = api.Problem(self.nel, self.mask, self.f, **args)
        return p

    def direct(self):
        return solve.solve_direct(self.K, self.mask, self.f)

    def compliance(self, u):
        return solve.compliance(self.f, u)

    def sensitivity(self, u):
        return solve.sensitivity(self.rho, u, self.nel, self.order, self.nsub, self.Ks, **MAT)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
