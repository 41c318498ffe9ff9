"""Partial diffusion approximation (Appendix A) -- FP64 CPU reference.

TEST INFRASTRUCTURE ONLY: the tests may use it; the product path never does.
It imports nothing from the HIP package.

Cells that the packets sample poorly get their temperature from the diffusion
approximation, div(D grad T^4) = 0 with D = 1 / (3 rho chi_R) (Appendix A),
with the well-sampled cells around them as boundary values.  The appendix
writes the discrete equation for a spherical-polar grid; on a Cartesian grid
the same construction reads, for a PDA cell c with face neighbours n along
axis a (cell size dx_a, Rosseland optical depth across a cell
dtau^a = rho chi_R dx_a):

    sum_a (1 / dx_a) sum_{n = c +- e_a} (u_n - u_c) / (dtau^a_n + dtau^a_c) = 0,  u = T^4,

i.e. conductances g_cn = 1 / (dx_a^2 (rho_c chi_R,c + rho_n chi_R,n)).  Readings:
  * PDA cells: dust cells whose absorption estimate is zero, or whose relative
    Monte-Carlo error exceeds `noise` (the paper's "fewer than a threshold of
    packets", measured by the estimator's own error);
  * a sampled dust neighbour is a boundary value (its T^4); an empty cell or
    the outside of the grid carries no flux;
  * chi_R is the Rosseland mean at the cell's current temperature; the linear
    system is solved `passes` times, chi_R re-evaluated at the new
    temperatures in between (Picard iteration);
  * a connected group of PDA cells without a sampled neighbour is left as it
    is (its system has no boundary value);
  * the new temperatures of PDA cells give their absorption rate by Eq. 3.
The linear solve is the library's sparse direct solver (scipy.sparse.linalg.spsolve).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components
from scipy.sparse.linalg import spsolve


def pda_cells(rho, adot, adot_sigma, noise):
    """mask of the cells the approximation takes over"""
    rho = np.asarray(rho).reshape(-1)
    adot = np.asarray(adot).reshape(-1)
    bad = adot <= 0.0
    if adot_sigma is not None:
        bad |= np.asarray(adot_sigma).reshape(-1) > noise * adot
    return (rho > 0.0) & bad


def _neighbours(n):
    """for each axis and direction: the neighbour's flat index (-1 outside)"""
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y, z = x.reshape(-1), y.reshape(-1), z.reshape(-1)
    out = []
    for a, (c, size) in enumerate(((x, nx), (y, ny), (z, nz))):
        stride = (1, nx, nx * ny)[a]
        for s in (-1, 1):
            ok = (c + s >= 0) & (c + s < size)
            out.append((a, np.where(ok, np.arange(x.size) + s * stride, -1)))
    return out


def solve_once(n, dx, rho, T, chi_r, pda):
    """one linear solve of the discrete diffusion equation on the PDA cells;
    returns the new temperatures and the mask of cells solved"""
    rho = np.asarray(rho, float).reshape(-1)
    T = np.asarray(T, float).reshape(-1)
    a = rho * np.asarray(chi_r, float).reshape(-1)
    idx = np.flatnonzero(pda)
    m = idx.size
    pos = -np.ones(rho.size, dtype=np.int64)
    pos[idx] = np.arange(m)
    diag = np.zeros(m)
    b = np.zeros(m)
    rows, cols, vals = [], [], []
    has_bc = np.zeros(m, bool)
    for ax, nb in _neighbours(n):
        nbc = nb[idx]
        ok = nbc >= 0
        ok[ok] = rho[nbc[ok]] > 0.0
        c = np.flatnonzero(ok)  # PDA cells (positions) with a dust neighbour here
        nn = nbc[c]
        g = 1.0 / (dx[ax] ** 2 * (a[idx[c]] + a[nn]))
        diag[c] += g
        inner = pda[nn]
        rows.append(c[inner])
        cols.append(pos[nn[inner]])
        vals.append(-g[inner])
        b[c[~inner]] += g[~inner] * T[nn[~inner]] ** 4
        has_bc[c[~inner]] = True
    A = sp.csr_matrix((np.concatenate(vals + [diag]),
                       (np.concatenate(rows + [np.arange(m)]), np.concatenate(cols + [np.arange(m)]))),
                      shape=(m, m))
    # solvable: connected groups of PDA cells with at least one boundary value
    ncomp, lab = connected_components(A, directed=False)
    good = np.zeros(ncomp, bool)
    good[np.unique(lab[has_bc])] = True
    keep = good[lab]
    Tn = T.copy()
    solved = np.zeros(rho.size, bool)
    if keep.any():
        k = np.flatnonzero(keep)
        u = spsolve(A[k][:, k].tocsc(), b[k])
        Tn[idx[k]] = u ** 0.25
        solved[idx[k]] = True
    return Tn, solved


def apply(model, noise: float, passes: int = 3):
    """the approximation on an oracle model after an iteration: new T and
    Adot of the PDA cells; returns (T, Adot, mask of solved cells)"""
    n = model.cfg["grid"]["n"]
    lo = np.asarray(model.cfg["grid"]["lo"], float)
    hi = np.asarray(model.cfg["grid"]["hi"], float)
    dx = (hi - lo) / np.asarray(n, float)
    rho = np.asarray(model.cfg["rho"], float).reshape(-1)
    adot, sig = model.specific_energy(with_sigma=True)
    T = model.temperature()
    pda = pda_cells(rho, adot, sig if model.run.get("want_noise", 0) else None, noise)
    # chi_R is needed on the PDA cells and their dust neighbours
    need = pda.copy()
    for _, nb in _neighbours(n):
        k = nb[pda]
        need[k[k >= 0]] = True
    need &= rho > 0.0
    solved = np.zeros(rho.size, bool)
    for _ in range(passes):
        chi_r = np.zeros(rho.size)
        for j in np.flatnonzero(need):
            chi_r[j] = model.rosseland_chi(T[j])
        T, solved = solve_once(n, dx, rho, T, chi_r, pda)
    adot = adot.copy()
    for j in np.flatnonzero(solved):
        adot[j] = model.adot_of_T(T[j])
    return T, adot, solved
