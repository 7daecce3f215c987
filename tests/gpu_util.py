"""Helpers shared by the GPU tests: the library handle and the oracle for
the same seeded problem, and comparisons."""
import numpy as np

from paper_2010_04559_amd import inputs
from oracle_problem import OracleProblem


def torch_mod():
    import torch
    return torch


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def to_dev(x, dtype=None):
    torch = torch_mod()
    return torch.as_tensor(np.asarray(x), dtype=dtype or torch.float64, device="cuda").contiguous()


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


class Pair:
    """The HIP library and the oracle set up for one problem."""

    def __init__(self, prob, with_mg=True):
        from paper_2010_04559_amd.transport import Transport
        self.prob = prob
        self.tr = Transport(prob)
        self.op = OracleProblem(prob, with_mg=with_mg)

    def level(self, l, outer=False):
        if outer:
            return self.op.outer
        return self.op.mg.levels[l]


def small(dim=2, n=3, level=1, order=4, g=0.8, c=0.9, seed=0, **kw):
    return inputs.small_problem(dim=dim, n=n, level=level, g=g, order=order, c=c, seed=seed, **kw)
