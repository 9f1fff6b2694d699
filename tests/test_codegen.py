"""Host-only checks of the run-time specialiser: the generated kernel source
(multivariate Horner scheme, power forms, batch entry) compiles for gfx950
with hiprtc for each form of integrand.  Numerics are the GPU parity tests'."""

import pytest

import paper_1811_11720_amd as Q
import workloads as W

KOR3 = (W.T_KOROBOV, 3, 3)


@pytest.mark.parametrize("case", ["sector_real", "signed_half_integer", "plain_product", "large_polynomial",
                                  "complex_sector"])
def test_specialised_source_compiles(case):
    if case == "sector_real":  # bounded U, F: one reciprocal square root for both powers
        desc, tr = W.sector_real(), KOR3
    elif case == "signed_half_integer":  # negative coefficients: separate powers
        desc = W.monomial([3.0, -1.0, 1.0, 2.0, 1.0, -1.0],
                          [[0, 0, 0], [1, 1, 0], [0, 0, 2], [0, 0, 0], [1, 0, 0], [0, 1, 1]], 3, n_u=3,
                          pow_u=-1.5, pow_f=-2.5)
        tr = (W.T_BAKER, 0, 0)
    elif case == "plain_product":  # F = 1, integer power
        desc, tr = W.plain_product(seed=1), KOR3
    elif case == "large_polynomial":  # more terms than the exhaustive split search takes at once
        desc, tr = W.random_real_small(seed=5, dim=12, n_u=20, n_f=60), (W.T_SIDI, 3, 0)
    else:
        desc, tr = W.sector_complex(), KOR3
    assert Q.specialize_check(desc, tr) > 1000
