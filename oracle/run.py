"""Time marching with the five sub-steps of Sec. 2.5, FP64.

Test infrastructure only (see oracle/__init__.py).
"""
from . import ib, lbm
from .lattice import for_dim


class Simulation:
    """Grid + optional immersed body, stepped with the paper's per-step procedure."""

    def __init__(self, D, dims, prm, state=None):
        self.lat = for_dim(D)
        self.prm = prm
        self.dims = tuple(dims)
        grid = tuple(dims[::-1])
        self.st = state if state is not None else lbm.freestream_state(self.lat, prm, grid)
        self.geom = None
        self.mk = None
        self.last_markers = None

    def set_markers(self, X, n, u_wall, t_kind, t_value, method=ib.FODIBM_R, kernel=ib.KERNEL_COS):
        self.geom = ib.build_geometry(self.dims, X, n, method, kernel)
        self.mk = ib.Markers(u_wall=u_wall, t_kind=t_kind, t_value=t_value)

    def step(self, n=1):
        for _ in range(n):
            if self.geom is not None:
                fib, fE, mf = ib.ib_step_forcing(self.lat, self.prm, self.geom, self.mk, self.st)
                self.last_markers = mf
            else:
                fib = fE = None
            self.st = lbm.lbm_step(self.lat, self.prm, self.st, fib, fE)
        return self.st

    def fields(self):
        return lbm.fields(self.lat, self.prm, self.st)
