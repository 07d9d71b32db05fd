"""Static grid refinement (ratio 2): fine blocks embedded in a coarse grid, 2D or 3D, nested to any depth.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs every experiment on locally refined meshes and does not state its refinement
scheme; this module writes out the one this project adopts, so that the GPU coupling can be
checked element by element. Readings (acoustic scaling, as for lattice Boltzmann multi-grid
methods in general):
  * fine node 2k along axis a coincides with coarse node origin[a] + k; the fine grid spacing and
    time step are half the coarse ones, so velocities, density and temperature keep their lattice
    values, and the fine viscosity and conductivity in lattice units are twice the coarse ones;
  * per coarse step the coarse grid steps first, then the fine block takes two steps; after each
    one its outer band (G fine nodes wide) is refilled from the coarse grid, interpolated
    multilinearly in space and linearly in time (weight 1/2, then 1);
  * a transferred population keeps the equilibrium of its own macros (Eq. (A.3)) and scales its
    non-equilibrium part by s = taubar_f / (2 taubar_c) coarse to fine, 1/s fine to coarse
    (taubar = mu / (rho cs^2) + 1/2 of each level at the local density); rho E is transferred as
    it is; of the force history H2, a per-step rate, the diagonal (trace-free) part scales by 1/2
    and 2; the off-diagonal part, which the scheme produces only where a level's own body forces,
    is not transferred (each level keeps what its own step produced);
  * after the fine steps, the coarse nodes whose fine counterpart lies at least R fine nodes inside
    the block on every axis take the fine values (restriction); the coarse grid is stepped
    everywhere;
  * levels nest: a block may itself hold a finer block, coupled to it in the same way, so that
    level k takes 2^k steps per step of level 0; a body lies on the finest level.
The coupling is not conservative (interpolation, not flux matching).
"""
import itertools
from dataclasses import dataclass, replace

import numpy as np

from oracle import lbm as L


@dataclass
class Block:
    origin: tuple   # coarse node of fine node 0, per axis (x, y[, z])
    size: tuple     # extent in coarse cells per axis: the fine grid has 2 size[a] nodes on axis a
    G: int = 2      # band refilled from the coarse grid (fine nodes; two cover one fine step's reach)
    R: int = 8      # restriction margin (fine nodes)

    @property
    def D(self):
        return len(self.size)

    @property
    def fine_dims(self):
        """Fine node counts per axis (x, y[, z])."""
        return tuple(2 * s for s in self.size)

    @property
    def fine_shape(self):
        """Array shape of a fine scalar field (x fastest)."""
        return tuple(reversed(self.fine_dims))


def fine_params(prm_c):
    """The fine level's parameters: viscosity and conductivity doubled in lattice units; its
    edges are refilled, so its own wrap is periodic."""
    return replace(prm_c, mu=2.0 * prm_c.mu, lam=2.0 * prm_c.lam, bc='periodic')


def _taubar(prm, rho):
    return prm.mu / (rho * (1.0 / 3.0)) + 0.5


def _rescale(lat, prm, f, rhoE, factor_of_rho):
    """f -> f^eq(its macros) + factor(rho) (f - f^eq)."""
    rho, _, u, T = L.predicted_macros(lat, prm, f, rhoE)
    feq = L.equilibrium(lat, rho, u, T)
    return feq + factor_of_rho(rho) * (f - feq)


def _open(idx, D):
    """Open-mesh index of per-axis index lists (x first) into an array with x on the last axis."""
    return np.ix_(*reversed(idx))


def band_mask(block):
    """Fine nodes within G of an edge of the block on some axis."""
    D, G = block.D, block.G
    m = np.zeros(block.fine_shape, dtype=bool)
    for a in range(D):
        n = block.fine_dims[a]
        x = np.arange(n)
        shape = [1] * D
        shape[D - 1 - a] = n
        m |= ((x < G) | (x >= n - G)).reshape(shape)
    return m


def interpolate(block, arr):
    """Multilinear interpolation of coarse fields arr [..., *coarse grid] at every fine node."""
    D = block.D
    shape_c = arr.shape[arr.ndim - D:]
    lo, hi, frac = [], [], []
    for a in range(D):
        n = block.fine_dims[a]
        nc = shape_c[D - 1 - a]
        xf = np.arange(n)
        i0 = block.origin[a] + xf // 2
        lo.append(i0 % nc)
        hi.append((i0 + 1) % nc)
        frac.append((xf % 2) * 0.5)
    out = 0.0
    for corner in itertools.product((0, 1), repeat=D):
        wt = 1.0
        for a in range(D):
            shape = [1] * D
            shape[D - 1 - a] = -1
            wt = wt * (frac[a] if corner[a] else 1.0 - frac[a]).reshape(shape)
        idx = [hi[a] if corner[a] else lo[a] for a in range(D)]
        out = out + wt * arr[(Ellipsis,) + _open(idx, D)]
    return out


def prolong(lat, prm_c, prm_f, f_c, e_c, H2_c, block):
    """Values at every fine node from a coarse state, rescaled to the fine level: populations
    [Q, *fine], rho E [*fine], diagonal H2 [D, *fine] (H2_f[a, a])."""
    D = block.D
    f = interpolate(block, f_c)
    e = interpolate(block, e_c)
    H2d = 0.5 * np.stack([interpolate(block, H2_c[a, a]) for a in range(D)])
    f = _rescale(lat, prm_c, f, e, lambda rho: _taubar(prm_f, rho) / (2.0 * _taubar(prm_c, rho)))
    return f, e, H2d


def fill_band(lat, prm_c, prm_f, st_f, st_a, st_b, wt, block):
    """Refill the fine band from the coarse state (1 - wt) a + wt b."""
    f_c = (1.0 - wt) * st_a.f + wt * st_b.f
    e_c = (1.0 - wt) * st_a.rhoE + wt * st_b.rhoE
    H2_c = (1.0 - wt) * st_a.H2 + wt * st_b.H2
    f, e, H2d = prolong(lat, prm_c, prm_f, f_c, e_c, H2_c, block)
    m = band_mask(block)
    st_f.f[:, m] = f[:, m]
    st_f.rhoE[m] = e[m]
    for a in range(block.D):
        st_f.H2[a, a][m] = H2d[a][m]
    rho, _, _, T = L.predicted_macros(lat, prm_f, st_f.f, st_f.rhoE)
    st_f.H1[m] = (rho * (1.0 - T))[m]
    return st_f


def restriction_nodes(block):
    """Per axis: the fine indices 2k at least R inside the block, and their coarse nodes."""
    fine, coarse = [], []
    for a in range(block.D):
        n = block.fine_dims[a]
        i = np.arange(0, n, 2)
        i = i[(i >= block.R) & (i <= n - 1 - block.R)]
        fine.append(i)
        coarse.append(block.origin[a] + i // 2)
    return fine, coarse


def restrict(lat, prm_c, prm_f, st_c, st_f, block):
    """Coarse nodes inside the block take the fine values of their coinciding fine nodes."""
    D = block.D
    fi, ci = restriction_nodes(block)
    sf, sc = _open(fi, D), _open(ci, D)
    f = st_f.f[(slice(None),) + sf]
    e = st_f.rhoE[sf]
    f = _rescale(lat, prm_f, f, e, lambda rho: 2.0 * _taubar(prm_c, rho) / _taubar(prm_f, rho))
    st_c.f[(slice(None),) + sc] = f
    st_c.rhoE[sc] = e
    for a in range(D):
        st_c.H2[a, a][sc] = 2.0 * st_f.H2[a, a][sf]
    rho, _, _, T = L.predicted_macros(lat, prm_c, st_c.f[(slice(None),) + sc], st_c.rhoE[sc])
    st_c.H1[sc] = rho * (1.0 - T)
    return st_c


def nested_step(lat, prm_0, states, blocks, finest_forcing=None):
    """One step of level 0 of nested blocks: level k + 1 lies in level k at blocks[k] and takes two
    steps per step of level k, each followed by its band refill from level k, and restricts onto
    level k at the end of level k's step (so level k takes 2^k steps per step of level 0). A body,
    if any, is on the finest level: finest_forcing(state) -> (fib, fE). Returns the new states,
    coarsest first."""
    states = list(states)

    def advance(k, prm):
        if k == len(states) - 1:
            fib, fE = finest_forcing(states[k]) if finest_forcing else (None, None)
            states[k] = L.lbm_step(lat, prm, states[k], fib, fE)
            return
        old = states[k]
        new = L.lbm_step(lat, prm, old)
        states[k] = new
        prm_f = fine_params(prm)
        for s in (1, 2):
            advance(k + 1, prm_f)
            states[k + 1] = fill_band(lat, prm, prm_f, states[k + 1], old, new, 0.5 * s, blocks[k])
        states[k] = restrict(lat, prm, prm_f, states[k], states[k + 1], blocks[k])

    advance(0, prm_0)
    return states


def refined_step(lat, prm_c, st_c, st_f, block, fine_forcing=None):
    """One coarse step of the two-level grid. fine_forcing(st_f) -> (fib, fE) of the fine body
    (None: no body). Returns the new coarse and fine states."""
    new_c, new_f = nested_step(lat, prm_c, [st_c, st_f], [block], fine_forcing)
    return new_c, new_f


def initial_nest(lat, prm_0, st_0, blocks):
    """States of every level of a nest, each finer one prolonged from the one containing it."""
    states, prm = [st_0], prm_0
    for blk in blocks:
        states.append(initial_fine(lat, prm, states[-1], blk))
        prm = fine_params(prm)
    return states


def initial_fine(lat, prm_c, st_c, block):
    """A fine state prolonged from a coarse state at every fine node (no off-diagonal history)."""
    prm_f = fine_params(prm_c)
    D = block.D
    f, e, H2d = prolong(lat, prm_c, prm_f, st_c.f, st_c.rhoE, st_c.H2, block)
    rho, _, _, T = L.predicted_macros(lat, prm_f, f, e)
    H2 = np.zeros((D, D) + block.fine_shape)
    for a in range(D):
        H2[a, a] = H2d[a]
    return L.State(f=f, rhoE=e, H1=rho * (1.0 - T), H2=H2)
