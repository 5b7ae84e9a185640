"""The paper's printed ion-acoustic parameters (tests/golden/iaw_parameters.json,
Sec. 4.1) against the units this implementation uses.

Lengths here are in Debye lengths lambda_D = v_th,e / omega_pe and times in
1/omega_pi, so the ion sound speed c_s = lambda_D omega_pi is 1.  The paper's
numbers must satisfy that identity, its stated step and grid ratios, and the
oracle's Boltzmann-electron dispersion relation must give the sound speed at the
paper's wave number.
"""
import json
import math
import os

import numpy as np

from oracle import pic
from oracle.pic import Grid

HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    with open(os.path.join(HERE, "golden", "iaw_parameters.json")) as f:
        return json.load(f)


def test_plasma_frequency_ratio_is_mass_ratio():
    g = golden()
    ratio = g["omega_pe"] / g["omega_pi"]
    assert abs(ratio - math.sqrt(abs(g["q_over_m_electron"] / g["q_over_m_ion"]))) < 1e-3 * ratio


def test_stated_step_and_grid_ratios():
    g = golden()
    assert abs(g["dt"] * g["omega_pe"] - g["dt_times_omega_pe_stated"]) < 0.02 * 0.25
    debye = g["v_th_electron"] / g["omega_pe"]
    assert abs(g["h"] / debye - g["h_over_debye_stated"]) < 0.01 * 0.28


def test_sound_speed_is_one_in_debye_and_ion_plasma_units():
    g = golden()
    debye = g["v_th_electron"] / g["omega_pe"]
    c_s = debye * g["omega_pi"]  # sqrt(T_e / m_i) in the paper's code units
    assert abs(c_s - 1.0) < 0.01


def test_oracle_dispersion_at_the_papers_wave_number():
    """Cold-ion Boltzmann-electron waves of the oracle (eq. 3.15 linearised)
    propagate at c_s / sqrt(1 + k^2) (units of lambda_D and omega_pi); at the
    paper's k lambda_D for L = 4 that is the sound speed to 0.1 %."""
    g = golden()
    debye = g["v_th_electron"] / g["omega_pe"]
    k = 2.0 * math.pi / g["domain_lengths"][0] * debye  # k lambda_D
    # discrete operator of the oracle on a fine grid: omega^2 = K^2 / (1 + K^2)
    grid = Grid(4096, 4096 * 0.05)
    h = grid.h
    K2 = (4.0 / h ** 2) * math.sin(k * h / 2.0) ** 2
    omega = math.sqrt(K2 / (1.0 + K2))
    assert abs(omega / k - 1.0) < 1e-3
    # the oracle's own Laplacian has the eigenvalue K^2 on that mode
    L = pic.neg_laplacian(grid)
    x = np.arange(grid.n_cells) * h
    kk = 2.0 * math.pi * 7 / grid.length
    mode = np.cos(kk * x)
    K2m = (4.0 / h ** 2) * math.sin(kk * h / 2.0) ** 2
    assert np.allclose(L @ mode, K2m * mode, rtol=0, atol=1e-9 * K2m)
