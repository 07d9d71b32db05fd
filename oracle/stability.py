"""Von Neumann analysis of the linearised hybrid LBM step, FP64, on the CPU.

Test and analysis infrastructure only (see oracle/__init__.py): it calls nothing but the
oracle's own step (lbm.lbm_step) and measures its linear response.

About a uniform free stream (rho_inf, u_inf, theta_inf; equilibrium populations, zero force
history) the step of Sec. 2.2 / Appendix A is translation invariant on a periodic grid, so a
perturbation e^{i k.x} v of the per-node state v is mapped to e^{i k.x} G(k) v. G(k) is measured
column by column: the state is perturbed by +-eps cos(k.x) v_j, stepped, and the Fourier
coefficients of the response at k give Re(G v_j) (cosine part) and -Im(G v_j) (sine part); the
central difference removes the quadratic terms. The scheme is linearly stable at k when every
eigenvalue of G(k) has modulus <= 1.

The MUSCL sign decisions of Eqs. (A.14)-(A.16) are piecewise linear in the velocity; with a
free-stream velocity component of at least the dead zone the decisions are fixed for small
perturbations and the step is linear in them. Along an axis where the free stream has no
velocity the decisions follow the perturbation's sign, and G is the derivative of one branch.

State per node: the Q populations, rho E, the force history H2 (deviatoric, symmetric: D(D+1)/2 - 1
components) and H1 (only read by the 'backward' reading of the time derivative in Eq. (A.9)).
"""
import numpy as np

from . import lbm
from .lattice import for_dim


def _basis(D):
    """Symmetric traceless D x D basis tensors of the force history."""
    out = []
    for a in range(D):
        for b in range(a + 1, D):
            t = np.zeros((D, D))
            t[a, b] = t[b, a] = 1.0
            out.append(t)
    for a in range(D - 1):
        t = np.zeros((D, D))
        t[a, a] = 1.0
        t[D - 1, D - 1] = -1.0
        out.append(t)
    return out


def amplification_matrix(prm, D, k, n=(16, 16, 16), eps=1e-7):
    """G(k) of the step about the free stream of prm on an n-periodic grid (n[a] nodes along
    axis a; k[a] = 2 pi m_a / n[a]). Returns G (complex, nv x nv) and the component names."""
    lat = for_dim(D)
    dims = tuple(int(n[a]) for a in range(D))
    grid = dims[::-1]
    base = lbm.freestream_state(lat, prm, grid)
    coords = np.meshgrid(*[np.arange(dims[a]) for a in range(D)], indexing='ij')
    phase = sum(k[a] * coords[a] for a in range(D)).transpose(tuple(range(D))[::-1])
    c, s = np.cos(phase), np.sin(phase)
    cc, ss = (c * c).sum(), (s * s).sum()
    hb = _basis(D)
    names = [f'f{i}' for i in range(lat.Q)] + ['rhoE'] + [f'H2_{j}' for j in range(len(hb))] + ['H1']
    nv = len(names)

    def pack(st):
        cols = [st.f[i] for i in range(lat.Q)] + [st.rhoE]
        cols += [(st.H2 * t.reshape((D, D) + (1,) * D)).sum(axis=(0, 1)) / (t * t).sum() for t in hb]
        cols += [st.H1]
        return cols

    def perturbed(j, amp):
        st = base.copy()
        d = amp * c
        if j < lat.Q:
            st.f = st.f.copy()
            st.f[j] = st.f[j] + d
        elif j == lat.Q:
            st.rhoE = st.rhoE + d
        elif j < nv - 1:
            t = hb[j - lat.Q - 1]
            st.H2 = st.H2 + t.reshape((D, D) + (1,) * D) * d
        else:
            st.H1 = st.H1 + d
        return st

    G = np.zeros((nv, nv), dtype=complex)
    for j in range(nv):
        plus = pack(lbm.lbm_step(lat, prm, perturbed(j, eps)))
        minus = pack(lbm.lbm_step(lat, prm, perturbed(j, -eps)))
        for i in range(nv):
            d = (plus[i] - minus[i]) / (2.0 * eps)
            re = (d * c).sum() / cc
            im = -(d * s).sum() / ss if ss > 0 else 0.0
            G[i, j] = re + 1j * im
    return G, names


def spectral_radius(prm, D, k, n=(16, 16, 16), active_h1=None):
    """Largest |eigenvalue| of G(k). The H1 component is dropped unless the time derivative of
    Eq. (A.9) reads it (prm.dt_form == 'backward'); otherwise it is a decoupled unit eigenvalue."""
    G, names = amplification_matrix(prm, D, k, n)
    use_h1 = prm.dt_form == 'backward' if active_h1 is None else active_h1
    if not use_h1:
        G = G[:-1, :-1]
    return float(np.abs(np.linalg.eigvals(G)).max())


def directions(D):
    """Wave directions checked: the axes and the in-plane diagonals (unit integer vectors)."""
    if D == 2:
        return [(1, 0), (0, 1), (1, 1), (1, -1)]
    return [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1)]


def max_growth(prm, D, n=16, modes=None):
    """max over wave directions and wavenumbers m = 1 .. n/2 - 1 along each direction of the
    spectral radius of G(k). Returns (radius, k of the worst mode)."""
    worst, kw = 0.0, None
    ms = range(1, n // 2) if modes is None else modes
    for dvec in directions(D):
        dims = tuple(n if dvec[a] else 2 for a in range(D))     # uniform along axes the wave misses
        for m in ms:
            k = [2.0 * np.pi * m * dvec[a] / n for a in range(D)]
            r = spectral_radius(prm, D, k, dims)
            if r > worst:
                worst, kw = r, tuple(k)
    return worst, kw


__all__ = ['amplification_matrix', 'spectral_radius', 'directions', 'max_growth']
