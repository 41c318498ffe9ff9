"""Pins of the oracle's partial diffusion approximation (Appendix A).

* A column of PDA cells between two sampled cells, uniform density: T^4 is
  linear between the boundary cells' centres (the discrete diffusion equation
  has the continuous solution).
* Two materials along the column: T^4 is linear in the Rosseland optical depth
  between cell centres (constant flux), so it kinks where the material changes
  (a conductance built from the wrong density or cell size fails).
* A cube whose shell is sampled at one temperature: the interior takes it.
* Empty cells carry no flux (the two halves of a column split by an empty
  cell each take their own boundary's temperature); a group with no sampled
  neighbour is left as it is.
* The selection: zero absorption or relative error above the threshold.
"""
import numpy as np
import pytest

from oracle import pda


def _line(nx, a_cells, T_left, T_right):
    n = (nx, 1, 1)
    dx = np.array([2.0, 1.0, 1.0])
    rho = np.ones(nx)
    chi = np.asarray(a_cells, float)  # rho = 1: a = chi
    T = np.full(nx, 10.0)
    T[0], T[-1] = T_left, T_right
    mask = np.zeros(nx, bool)
    mask[1:-1] = True
    return n, dx, rho, T, chi, mask


def test_uniform_column_is_linear_in_T4():
    nx = 12
    n, dx, rho, T, chi, mask = _line(nx, np.full(nx, 3.0), 100.0, 20.0)
    Tn, solved = pda.solve_once(n, dx, rho, T, chi, mask)
    assert solved[1:-1].all() and not solved[0] and not solved[-1]
    u = 100.0 ** 4 + (20.0 ** 4 - 100.0 ** 4) * np.arange(nx) / (nx - 1)
    np.testing.assert_allclose(Tn ** 4, u, rtol=1e-12)


def test_two_materials_linear_in_optical_depth():
    nx = 10
    a = np.where(np.arange(nx) < 4, 1.0, 7.0)
    n, dx, rho, T, chi, mask = _line(nx, a, 300.0, 40.0)
    Tn, _ = pda.solve_once(n, dx, rho, T, chi, mask)
    # optical depth between centres j, j+1: (a_j + a_{j+1}) dx / 2
    tau = np.concatenate([[0.0], np.cumsum((a[:-1] + a[1:]) * dx[0] / 2)])
    u = 300.0 ** 4 + (40.0 ** 4 - 300.0 ** 4) * tau / tau[-1]
    np.testing.assert_allclose(Tn ** 4, u, rtol=1e-12)
    slope = np.diff(Tn ** 4)
    # constant flux: a cell of the dense material drops T^4 seven times as much
    assert slope[6] / slope[1] == pytest.approx(7.0, rel=1e-9)


def test_cube_interior_takes_the_shell_temperature():
    m = 6
    n = (m, m, m)
    dx = np.array([1.0, 2.0, 0.5])
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, m ** 3)
    chi = rng.uniform(1.0, 5.0, m ** 3)
    T = rng.uniform(5.0, 50.0, m ** 3)
    z, y, x = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    shell = ((x == 0) | (x == m - 1) | (y == 0) | (y == m - 1) | (z == 0) | (z == m - 1)).reshape(-1)
    T[shell] = 77.0
    Tn, solved = pda.solve_once(n, dx, rho, T, chi, ~shell)
    assert solved[~shell].all()
    np.testing.assert_allclose(Tn, 77.0, rtol=1e-12)


def test_empty_cells_and_isolated_groups():
    nx = 9
    n, dx, rho, T, chi, mask = _line(nx, np.full(nx, 2.0), 50.0, 90.0)
    rho[4] = 0.0  # an empty cell splits the column
    mask[4] = False
    Tn, solved = pda.solve_once(n, dx, rho, T, chi, mask)
    np.testing.assert_allclose(Tn[1:4], 50.0, rtol=1e-12)
    np.testing.assert_allclose(Tn[5:8], 90.0, rtol=1e-12)
    # no sampled neighbour at all: unchanged, not solved
    n, dx, rho, T, chi, mask = _line(nx, np.full(nx, 2.0), 50.0, 90.0)
    rho[0] = rho[-1] = 0.0
    Tn, solved = pda.solve_once(n, dx, rho, T, chi, mask)
    assert not solved.any()
    np.testing.assert_array_equal(Tn, T)


def test_selection():
    rho = np.array([1.0, 1.0, 1.0, 0.0, 1.0])
    adot = np.array([1.0, 0.0, 2.0, 0.0, 5.0])
    sig = np.array([0.05, 0.0, 0.5, 0.0, 0.2])
    np.testing.assert_array_equal(pda.pda_cells(rho, adot, sig, 0.1), [False, True, True, False, False])
    np.testing.assert_array_equal(pda.pda_cells(rho, adot, None, 0.1), [False, True, False, False, False])
