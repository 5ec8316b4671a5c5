"""Host pieces of the sweep tool and the damping switch (no GPU work)."""
import numpy as np

from oracle import jackson, metrics


def test_sweep_ari_matches_oracle_metric():
    from paper_1602_02018_amd import sweeps

    rng = np.random.default_rng(0)
    for _ in range(20):
        a = rng.integers(0, 5, 200)
        b = np.where(rng.random(200) < 0.7, a, rng.integers(0, 5, 200))
        assert abs(sweeps.ari(a, b) - metrics.adjusted_rand_index(a, b)) < 1e-12
    assert sweeps.ari([0, 0, 1, 1], [3, 3, 7, 7]) == 1.0


def test_damping_switch_changes_host_coefficients():
    from paper_1602_02018_amd import _lib, api

    try:
        assert api.get_damping() == _lib.DAMP_JACKSON
        np.testing.assert_allclose(api.jackson_coeffs(0.4, 30), jackson.lowpass_coeffs(0.4, 30),
                                   rtol=1e-13, atol=1e-15)
        api.set_damping(_lib.DAMP_NONE)
        np.testing.assert_allclose(api.jackson_coeffs(0.4, 30),
                                   jackson.lowpass_coeffs(0.4, 30, damping=False),
                                   rtol=1e-13, atol=1e-15)
        assert _lib.lib().csc_set_damping(7) == _lib.CSC_E_INVALID_ARG
    finally:
        api.set_damping(_lib.DAMP_JACKSON)
