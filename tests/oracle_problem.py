"""Builds the oracle's objects for a seeded problem description.

Test infrastructure: it turns a ``Problem`` from the input generators into
the oracle's grid, angular mesh, outer level (full scatter order), V-cycle
levels, right-hand side and detector weights.  Only tests and the benchmark's
CPU-baseline leg use it.
"""
import numpy as np

from oracle import angular as ang
from oracle import spatial as sp
from oracle import transport as tr
from oracle import multigrid as mgm


def angular_mesh(spec):
    if spec.band_lmax > 0:
        return ang.AngularMesh.band_z(spec.band_lmax)
    if spec.extra_levels > 0:
        return ang.AngularMesh.cone(spec.cone_axis, spec.cone_half_angle_deg, spec.base_level,
                                    spec.extra_levels, closure=spec.closure)
    return ang.AngularMesh.uniform(spec.base_level)


class OracleProblem:
    def __init__(self, prob, with_mg=True):
        self.prob = prob
        self.grid = sp.Grid(prob.dim, prob.n, prob.length)
        self.mesh = angular_mesh(prob.angular)
        self.T = self.mesh.levels()
        basis = getattr(prob.angular, "basis", "lin")
        self.outer = tr.Level(self.grid, self.T[-1], prob.sigma_t, prob.sigma_s, prob.moments(), basis=basis)
        self.mg = None
        if with_mg:
            full = prob.moments(max(prob.mg_orders))
            self.mg = mgm.AngularMG(self.grid, self.mesh, prob.sigma_t, prob.sigma_s, full,
                                    prob.mg_orders, prob.nu_pre, prob.nu_post, prob.nu_coarse,
                                    octant_order=prob.octant_order, basis=basis)

    def rhs(self):
        p, lv = self.prob, self.outer
        b = lv.rhs_volume(p.q_cell)
        f = p.inflow
        if f is not None:
            if f.kind == "iso":
                b = b + lv.rhs_inflow_iso(f.axis, f.side, f.lo, f.hi, f.value)
            else:
                b = b + lv.rhs_beam(f.direction, f.axis, f.side, f.lo, f.hi, f.value)
        return b

    def detector(self):
        lo, hi = self.prob.detector
        return self.outer.detector_weights(lo, hi)
