"""Self-consistency of the exact results the oracle is checked against.

Enumeration, the transfer matrix and Kaufman's closed form must agree on small
tori; Onsager's energy and Yang's magnetisation must hit their known limits;
the paper's printed critical temperature (section 3.1) must agree with
2/ln(1+sqrt 2) to the printed digits.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import signal

from oracle import exact, stats

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_printed_tc_matches_onsager():
    with open(os.path.join(GOLD, "paper_values.json")) as f:
        v = json.load(f)["critical_temperature"]["value"]
    assert abs(exact.T_C - v) < 5e-7
    assert abs(exact.T_C - 2.0 / math.log(1.0 + math.sqrt(2.0))) == 0.0


@pytest.mark.parametrize("T", [1.3, exact.T_C, 3.7])
def test_enumeration_equals_transfer_and_kaufman_4x4(T):
    B, _ = exact.enumerate_torus(4, 4)
    a = B.astype(np.float64) / T
    lz = a.max() + math.log(np.exp(a - a.max()).sum())
    assert abs(lz - exact.transfer_lnZ(4, 4, 1 / T)) < 1e-10
    assert abs(lz - float(exact.kaufman_lnZ(4, 4, 1 / T))) < 1e-10
    e_enum, _ = exact.enum_moments(4, 4, T)
    assert abs(e_enum - exact.kaufman_energy(4, 4, T)) < 1e-10


@pytest.mark.parametrize("n,m", [(4, 6), (6, 4), (4, 8), (8, 6), (2, 10)])
def test_kaufman_equals_transfer(n, m):
    for T in (1.7, exact.T_C, 2.9):
        assert abs(float(exact.kaufman_lnZ(n, m, 1 / T)) - exact.transfer_lnZ(n, m, 1 / T)) < 1e-9
        assert abs(float(exact.kaufman_lnZ(n, m, 1 / T)) - exact.transfer_lnZ(m, n, 1 / T)) < 1e-9


def test_kaufman_approaches_onsager():
    # finite-size corrections at T = 2.0 (xi ~ 1) are exponentially small
    assert abs(exact.kaufman_energy(128, 128, 2.0) - exact.onsager_u(2.0)) < 1e-10
    # at T_c the finite-size energy approaches -sqrt2 from below as 1/L
    e = [exact.kaufman_energy(L, L, exact.T_C) for L in (16, 32, 64)]
    assert e[0] < e[1] < e[2] < -math.sqrt(2)
    assert abs((e[1] + math.sqrt(2)) / (e[0] + math.sqrt(2)) - 0.5) < 0.05


def test_onsager_limits():
    assert abs(exact.onsager_u(0.05) + 2.0) < 1e-12          # ground state: 2 bonds per spin
    assert abs(exact.onsager_u(1e4)) < 1e-3                   # high T: u -> -2 tanh(1/T) -> 0
    assert abs(exact.onsager_u(200.0) + 2 * math.tanh(1 / 200.0)) < 1e-4
    # continuity through T_c
    # (u - u_c ~ (T - T_c) ln|T - T_c|, so a 1e-6 step moves u by about 1e-5)
    assert abs(exact.onsager_u(exact.T_C * (1 + 1e-6)) + math.sqrt(2)) < 1e-4
    assert abs(exact.onsager_u(exact.T_C * (1 - 1e-6)) + math.sqrt(2)) < 1e-4


def test_yang_limits():
    assert exact.yang_m(0.1) == pytest.approx(1.0, abs=1e-12)
    assert exact.yang_m(exact.T_C) == 0.0 and exact.yang_m(3.0) == 0.0
    # critical exponent 1/8: m ~ (T_c - T)^(1/8) near T_c
    t1, t2 = exact.T_C * (1 - 1e-6), exact.T_C * (1 - 1e-8)
    slope = math.log(exact.yang_m(t1) / exact.yang_m(t2)) / math.log(1e-6 / 1e-8)
    assert abs(slope - 0.125) < 1e-3


def test_tau_int_ar1_closed_form():
    # AR(1) with coefficient rho has tau_int = (1 + rho) / (2 (1 - rho))
    rng = np.random.default_rng(1)
    for rho in (0.0, 0.5, 0.9):
        n = 400000
        e = rng.standard_normal(n)
        x = signal.lfilter([1.0], [1.0, -rho], e)[1000:]
        tau, _ = stats.tau_int(x)
        exact_tau = (1 + rho) / (2 * (1 - rho))
        assert abs(tau - exact_tau) < 0.05 * exact_tau + 0.02, (rho, tau, exact_tau)


def test_table1_iteration_period_identity():
    # section 3.2 / Table 1: T_iter = n m N_sim / R_flip (R_flip rounded when printed)
    with open(os.path.join(GOLD, "paper_values.json")) as f:
        t1 = json.load(f)["table1"]
    for n, m, nsim, rflip, titer in t1["rows"]:
        t = n * m * nsim / rflip * 1e-6  # flip / (flip/ns) = ns -> ms
        assert abs(t - titer) / titer < 1e-3


def test_product_tau_estimator_matches_oracle_and_ar1():
    from paper_2404_16990_amd import analysis
    rng = np.random.default_rng(4)
    for rho in (0.3, 0.8, 0.95):
        x = signal.lfilter([1.0], [1.0, -rho], rng.standard_normal(300000))[2000:]
        t_prod, w_prod = analysis.tau_int(x)
        t_orc, w_orc = stats.tau_int(x)
        assert abs(t_prod - t_orc) < 1e-9 and w_prod == w_orc
        exact_tau = (1 + rho) / (2 * (1 - rho))
        assert abs(t_prod - exact_tau) < 0.06 * exact_tau
