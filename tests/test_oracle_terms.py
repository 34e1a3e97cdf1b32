"""Pins for the oracle's random numbers and pair potentials (CPU only).

Each check compares the oracle with something fixed outside it: published
known-answer vectors, closed-form well minima and zero crossings, limits of
the dielectric function, symmetry, and central finite differences.
"""
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
T = synth.TYPE_ID


def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert orc.philox(v[0:4], v[4:6]) == v[6:10]


def test_stream_word_layout(orc):
    # word w of (lig, run, gen, indiv, stream) is lane w%4 of the block w//4
    seed = (7 << 32) | 11
    out = orc.philox([5, 6, 7, (9 << 16) | (3 << 10) | 2], [11, 7])
    for lane in range(4):
        assert orc.stream_word(seed, 5, 6, 7, 9, 3, 8 + lane) == out[lane]


@pytest.mark.parametrize("ti,tj", [("C", "C"), ("C", "N"), ("A", "S"), ("N", "OA"), ("OA", "OA"),
                                   ("HD", "HD"), ("HD", "C"), ("NA", "SA")])
def test_vdw_well_depth_position_and_zero(orc, ff, ti, tj):
    i, j = T[ti], T[tj]
    R = 0.5 * (ff["Rii"][i] + ff["Rii"][j])
    eps = math.sqrt(ff["epsii"][i] * ff["epsii"][j])
    depth = -ff["w_vdw"] * eps
    # flat band of width `smooth` around the minimum
    for r in (R - 0.24, R, R + 0.24):
        e, d = orc.lj(i, j, r)
        assert e == pytest.approx(depth, rel=1e-12, abs=1e-15)
        assert d == 0.0
    # zero crossing of the 12-6 well at R / 2^(1/6), shifted out by smooth/2
    rz = R * 2 ** (-1 / 6) - ff["smooth"] / 2
    assert abs(orc.lj(i, j, rz)[0]) < 1e-12 * abs(ff["w_vdw"] * eps) * 1e3
    # symmetric in the two types
    assert orc.lj(i, j, 3.3)[0] == orc.lj(j, i, 3.3)[0]


@pytest.mark.parametrize("acc", ["OA", "NA", "SA"])
def test_hbond_only_between_donor_and_acceptor(orc, ff, acc):
    a, h = T[acc], T["HD"]
    Rhb, ehb = ff["Rhb"][a], ff["epshb"][a]
    e, d = orc.lj(h, a, Rhb)
    assert e == pytest.approx(-ff["w_hb"] * ehb, rel=1e-12)
    assert orc.lj(a, h, Rhb)[0] == e
    # 12-10 zero crossing at R_hb * sqrt(5/6), shifted by smooth/2
    rz = Rhb * math.sqrt(5 / 6) - ff["smooth"] / 2
    assert abs(orc.lj(h, a, rz)[0]) < 1e-9
    # acceptor-acceptor and donor-donor pairs keep the 12-6 well
    Ra = ff["Rii"][a]
    assert orc.lj(a, a, Ra)[0] == pytest.approx(-ff["w_vdw"] * ff["epsii"][a], rel=1e-12)
    assert orc.lj(h, h, ff["Rii"][h])[0] == pytest.approx(-ff["w_vdw"] * ff["epsii"][h], rel=1e-12)


def test_dielectric_limits(orc, ff):
    A, eps0, k = ff["diel_A"], ff["diel_eps0"], ff["diel_k"]
    B = eps0 - A
    assert orc.diel(0.0)[0] == pytest.approx(A + B / (1 + k), rel=1e-14)
    assert orc.diel(1e4)[0] == pytest.approx(eps0, rel=1e-14)
    # monotone increasing
    r = np.linspace(0.0, 40.0, 400)
    e = np.array([orc.diel(x)[0] for x in r])
    assert np.all(np.diff(e) > 0)
    # far field: Coulomb with the bulk dielectric
    for rr in (200.0, 500.0):
        val = orc.elec(0.3, -0.4, rr)[0]
        assert val == pytest.approx(ff["w_el"] * ff["coulomb"] * 0.3 * -0.4 / (eps0 * rr), rel=1e-12)


def test_desolvation_gaussian(orc, ff):
    i, j = T["C"], T["OA"]
    qi, qj = 0.2, -0.35
    Si = ff["solpar"][i] + ff["qasp"] * abs(qi)
    Sj = ff["solpar"][j] + ff["qasp"] * abs(qj)
    e0 = ff["w_sol"] * (Si * ff["vol"][j] + Sj * ff["vol"][i])
    # r = 0 is raised to the 0.01 A floor: exp(-1e-4 / (2 sigma^2)) differs from 1 by < 4e-6
    assert orc.desolv(i, qi, j, qj, 0.0)[0] == pytest.approx(e0, rel=5e-6)
    assert orc.desolv(i, qi, j, qj, 0.0)[0] == orc.desolv(i, qi, j, qj, ff['r_floor'])[0]
    rhalf = ff["sigma"] * math.sqrt(2 * math.log(2))
    assert orc.desolv(i, qi, j, qj, rhalf)[0] == pytest.approx(e0 / 2, rel=1e-12)
    assert orc.desolv(i, qi, j, qj, 3.0)[0] == orc.desolv(j, qj, i, qi, 3.0)[0]


def test_pair_is_sum_of_terms(orc):
    i, j = T["N"], T["HD"]
    for r in (0.5, 1.7, 2.9, 6.0):
        tot = orc.pair(i, 0.1, j, 0.25, r)[0]
        parts = orc.lj(i, j, r)[0] + orc.elec(0.1, 0.25, r)[0] + orc.desolv(i, 0.1, j, 0.25, r)[0]
        assert tot == pytest.approx(parts, rel=1e-14)


@pytest.mark.parametrize("ti,tj", [("C", "C"), ("HD", "OA"), ("N", "S")])
def test_pair_derivative_matches_finite_difference(orc, ti, tj):
    i, j = T[ti], T[tj]
    h = 1e-6
    for r in np.linspace(0.6, 9.0, 60):
        e, d = orc.pair(i, 0.17, j, -0.31, r)
        fd = (orc.pair(i, 0.17, j, -0.31, r + h)[0] - orc.pair(i, 0.17, j, -0.31, r - h)[0]) / (2 * h)
        assert d == pytest.approx(fd, rel=2e-6, abs=1e-7 * max(1.0, abs(e)))
