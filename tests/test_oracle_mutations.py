"""Planted mistakes in the oracle must fail its pins.

Each test swaps one step of the oracle (on the CPU, through monkeypatch) for a
version with a plausible slip - a dropped term, a wrong sign, a wrong index, a
transposed entry - and checks that the pin "p(l)-CG iterates equal CG iterates"
(used in test_oracle_pins.py) no longer holds.  This is what makes the pins
trustworthy: a mistake anywhere in the scalar or vector steps shows up.
"""
import numpy as np
import pytest

import synth
from oracle import cg as ocg
from oracle import operators, shifts
from oracle import plcg as oplcg


def _pin_holds(ls=(1, 2, 3), dots=("symmetric", "full")):
    A = operators.laplacian((16, 12))
    b = A(synth.uniform(A.n, 4))
    x0 = np.zeros(A.n)
    ref = ocg.cg(A, b, x0, 1e-30, 12, record_iterates=True)
    for l in ls:
        sig = shifts.chebyshev_shifts(l, 0.0, 8.0)
        for d in dots:
            r = oplcg.plcg(A, b, x0, l, sig, 1e-30, 12, dots=d, max_restarts=0)
            if r.iters != 12:
                return False
            if np.linalg.norm(r.x - ref.iterates[-1]) > 1e-10 * np.linalg.norm(ref.iterates[-1]):
                return False
    return True


def test_unmodified_oracle_passes():
    assert _pin_holds()


def _mut_fill_transposed(G, c, l):
    for j in range(max(0, c - 2 * l), c - l):
        G[j, c] = G[j + l, c - l] if (j + l, c - l) in G else 0.0


def _mut_finalize_no_correction(G, c, l):
    lo = max(0, c - 2 * l)
    for j in range(max(0, c - l + 1), c):
        G[j, c] = G[j, c] / G[j, j]
    arg = G[c, c] - sum(G[k, c] ** 2 for k in range(lo, c))
    if not arg > 0:
        raise oplcg.Breakdown(c - 1, "sqrt")
    G[c, c] = arg ** 0.5


def _mut_finalize_sum_off_by_one(G, c, l):
    lo = max(0, c - 2 * l)
    for j in range(max(0, c - l + 1), c):
        s = G[j, c]
        for k in range(lo, j - 1):          # drops the k = j-1 term
            s = s - G[k, j] * G[k, c]
        G[j, c] = s / G[j, j]
    arg = G[c, c] - sum(G[k, c] ** 2 for k in range(lo, c))
    if not arg > 0:
        raise oplcg.Breakdown(c - 1, "sqrt")
    G[c, c] = arg ** 0.5


def _mut_T_no_sigma(G, gam, dlt, sigma, t, l):
    corr = G[t - 1, t] * dlt[t - 1] if t >= 1 else 0.0
    if t < l:
        gam[t] = (G[t, t + 1] - corr) / G[t, t]
        dlt[t] = G[t + 1, t + 1] / G[t, t]
    else:
        gam[t] = (G[t, t] * gam[t - l] + G[t, t + 1] * dlt[t - l] - corr) / G[t, t]
        dlt[t] = (G[t + 1, t + 1] * dlt[t - l]) / G[t, t]


def _mut_T_wrong_lag(G, gam, dlt, sigma, t, l):
    corr = G[t - 1, t] * dlt[t - 1] if t >= 1 else 0.0
    if t < l:
        gam[t] = (G[t, t + 1] + sigma[t] * G[t, t] - corr) / G[t, t]
        dlt[t] = G[t + 1, t + 1] / G[t, t]
    else:
        gam[t] = (G[t, t] * gam[t - 1] + G[t, t + 1] * dlt[t - 1] - corr) / G[t, t]
        dlt[t] = (G[t + 1, t + 1] * dlt[t - 1]) / G[t, t]


def _mut_T_sign(G, gam, dlt, sigma, t, l):
    corr = G[t - 1, t] * dlt[t - 1] if t >= 1 else 0.0
    if t < l:
        gam[t] = (G[t, t + 1] + sigma[t] * G[t, t] + corr) / G[t, t]
        dlt[t] = G[t + 1, t + 1] / G[t, t]
    else:
        gam[t] = (G[t, t] * gam[t - l] + G[t, t + 1] * dlt[t - l] + corr) / G[t, t]
        dlt[t] = (G[t + 1, t + 1] * dlt[t - l]) / G[t, t]


def _mut_LU_zeta_sign(gam, dlt, eta, lam, zeta, t, beta):
    if t == 0:
        eta[0] = gam[0]
        zeta[0] = beta
    else:
        lam[t] = dlt[t - 1] / eta[t - 1]
        eta[t] = gam[t] - lam[t] * dlt[t - 1]
        zeta[t] = lam[t] * zeta[t - 1]


def _mut_basis_sigma_sign(z, gam, dlt, sigma, t, l, i, store=None):
    dm1 = dlt[t - 1] if t >= 1 else 0.0
    for k in range(l):
        new = z[k + 1][t + k + 1] - (sigma[k] - gam[t]) * z[k][t + k]
        if t >= 1:
            new = new - dm1 * z[k][t + k - 1]
        z[k][t + k + 1] = new / dlt[t]
    new = z[l][i + 1] - gam[t] * z[l][i]
    if t >= 1:
        new = new - dm1 * z[l][i - 1]
    z[l][i + 1] = new / dlt[t]


def _mut_basis_wrong_shift_index(z, gam, dlt, sigma, t, l, i, store=None):
    dm1 = dlt[t - 1] if t >= 1 else 0.0
    for k in range(l):
        new = z[k + 1][t + k + 1] + (sigma[l - 1 - k] - gam[t]) * z[k][t + k]
        if t >= 1:
            new = new - dm1 * z[k][t + k - 1]
        z[k][t + k + 1] = new / dlt[t]
    new = z[l][i + 1] - gam[t] * z[l][i]
    if t >= 1:
        new = new - dm1 * z[l][i - 1]
    z[l][i + 1] = new / dlt[t]


def _mut_dots_wrong_basis(G, z, i, l, dots, dot=np.dot):
    u = z[l][i + 1]
    c = i + 1
    j = i - l + 1
    if j >= 0:
        G[j, c] = np.dot(u, z[l][j])             # z^{(l)} instead of v = z^{(0)}
    for j in range(max(0, i - l + 2), i + 2):
        G[j, c] = np.dot(u, z[l][j])
    return l + 1


@pytest.mark.parametrize("name,fn,ls,dots", [
    ("fill_symmetric", _mut_fill_transposed, (2, 3), ("symmetric",)),
    ("finalize_column", _mut_finalize_no_correction, (2, 3), ("symmetric", "full")),
    ("finalize_column", _mut_finalize_sum_off_by_one, (2, 3), ("symmetric", "full")),
    ("update_T", _mut_T_no_sigma, (1, 2, 3), ("symmetric",)),
    ("update_T", _mut_T_wrong_lag, (2, 3), ("symmetric",)),
    ("update_T", _mut_T_sign, (1, 2, 3), ("symmetric",)),
    ("update_LU", _mut_LU_zeta_sign, (1, 2), ("symmetric",)),
    ("basis_updates", _mut_basis_sigma_sign, (1, 2, 3), ("symmetric",)),
    ("basis_updates", _mut_basis_wrong_shift_index, (2, 3), ("symmetric",)),
    ("start_dots", _mut_dots_wrong_basis, (1, 2, 3), ("symmetric",)),
])
def test_planted_mistake_is_caught(monkeypatch, name, fn, ls, dots):
    monkeypatch.setattr(oplcg, name, fn)
    assert not _pin_holds(ls, dots)
