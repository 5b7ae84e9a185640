"""The three-moment (EFREE) pins catch plausible mistakes: each case plants one in the
oracle (on the CPU, through monkeypatch) and checks that the pin written for that
part of the method then fails."""
import numpy as np
import pytest

from oracle import efpi
import test_oracle_efpi as pins


def _drop_mean_velocity(n_nodes, j_nodes, s_nodes, sch):
    # T = s / n instead of s / n - u^2
    n = np.maximum(np.asarray(n_nodes, dtype=np.float64), 0.0)
    s = np.asarray(s_nodes, dtype=np.float64)
    t = np.zeros_like(n)
    ok = n > sch.n_floor
    t[ok] = np.maximum(s[ok] / n[ok], 0.0)
    return t


def _mutations():
    restrict = efpi.restrict_snapshot
    correct = efpi.block_correct
    load = efpi.load_particles
    return [
        ("temperature without -u^2", "temperature_profile", _drop_mean_velocity,
         pins.test_temperature_profile_by_hand),
        ("moments of V instead of V~", "restrict_snapshot",
         lambda x, v, e, w, tau, g, lv, coev=True, moments=2:
         restrict(x, v, np.zeros_like(np.asarray(e, dtype=np.float64)), w, tau, g, lv, coev,
                  moments),
         pins.test_coevolving_moments_by_hand),
        ("no stretch to the second moment", "block_correct",
         lambda cell, v, w, coarse, g, sch: correct(cell, v, w, np.asarray(coarse)[:2], g, sch),
         pins.test_efree_block_correction_exact),
        ("thermal speed vth instead of sqrt(T)", "load_particles",
         lambda n, u, g, sch, shift, t_nodes=None: load(n, u, g, sch, shift, None),
         pins.test_load_particles_with_a_temperature_profile_by_hand),
    ]


@pytest.mark.parametrize("case", range(4))
def test_pin_fails_on_planted_mistake(case, monkeypatch):
    name, attr, bad, pin = _mutations()[case]
    pin()  # passes on the oracle as written
    monkeypatch.setattr(efpi, attr, bad)
    with pytest.raises(AssertionError):
        pin()
