"""Pins of the oracle against numbers the paper prints (golden fixtures).

Fig. 6 (Section 3.2) prints, for a 40 x 40 image with 100 angles of 40 rays,
kappa(W^T W) = 8.68e4 and, for the WTG-preconditioned operator, 3.42e2.  The
oracle's geometry (exact intersection lengths, angles k*pi/m, bins of one
pixel centred on the detector) and its multiplicative two-grid sweep with exact
coarse solves reproduce both to the printed three significant digits;
Joseph's kernel on the same geometry does not (it is about ten times worse
conditioned).
"""
import json
import os

import numpy as np
import pytest

from oracle import wmg
from oracle.geometry import Geometry
from oracle.projector import system_matrix

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_condition_numbers.json")))


def _sig3(v):
    return float(f"{v:.2e}")


@pytest.fixture(scope="module")
def system():
    g = Geometry(GOLD["n"], GOLD["angles"], GOLD["rays"])
    W = system_matrix(g)
    Wd = W.toarray()
    return g, W, Wd.T @ Wd


def test_kappa_unpreconditioned(system):
    _, _, A = system
    ev = np.linalg.eigvalsh(A)
    assert _sig3(ev.max() / ev.min()) == GOLD["kappa_unpreconditioned"]


def test_kappa_wavelet_two_grid(system):
    g, _, A = system
    cyc = wmg.WaveletCycle(A, g.n, 1, "multiplicative")
    Minv = np.column_stack([cyc(e) for e in np.eye(g.N)])
    ev = np.linalg.eigvals(A @ Minv)          # eq. spec_wavelet: I - A WTG A^-1 = A M^-1
    kappa = np.abs(ev).max() / np.abs(ev).min()
    assert _sig3(kappa) == GOLD["kappa_wtg"]


def test_packet_diagonal_reading_is_weaker_but_helps(system):
    """The additive packet-diagonal preconditioner (the scalable reading) lowers kappa,
    by less than the exact-solve cycle."""
    g, W, A = system
    d = wmg.packet_diagonal(W, g.n, 1)
    Minv = np.column_stack([wmg.apply_additive_diag(e, d, 1) for e in np.eye(g.N)])
    ev = np.linalg.eigvals(A @ Minv)
    kappa = np.abs(ev).max() / np.abs(ev).min()
    assert GOLD["kappa_wtg"] < kappa < GOLD["kappa_unpreconditioned"] / 2


def test_joseph_kernel_does_not_give_the_printed_spectrum():
    """Joseph's W on the same geometry: kappa(W^T W) about ten times the printed one."""
    from oracle import joseph
    g = Geometry(GOLD["n"], GOLD["angles"], GOLD["rays"])
    J = joseph.joseph_matrix(g).toarray()
    ev = np.linalg.eigvalsh(J.T @ J)
    kappa = ev.max() / ev.min()
    assert kappa > 5 * GOLD["kappa_unpreconditioned"], kappa
