"""CPU checks of the conditioned SPD recipe used by the conditioning parity
tests, and of the oracle on such inputs (Sec. III-C: scale and conditioning
are part of the validated contract)."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from paper_2609_28179_amd import inputs


@pytest.mark.parametrize("kappa", [1e2, 1e3, 1e4])
@pytest.mark.parametrize("n", [8, 33, 64])
def test_spd_conditioned_has_the_stated_spectrum(n, kappa):
    rng = inputs.rng_for(300, "posv", n, 4)
    A64 = inputs.spd_conditioned64(rng, 4, n, kappa)
    assert np.array_equal(A64, np.swapaxes(A64, 1, 2))
    lam = np.linalg.eigvalsh(A64)
    assert np.allclose(lam, np.logspace(0, np.log10(kappa), n)[None], rtol=1e-10)
    A32 = inputs.spd_conditioned(inputs.rng_for(300, "posv", n, 4), 4, n, kappa)
    assert np.array_equal(A32, A64.astype(np.float32))           # same draws
    c = np.linalg.cond(A32.astype(np.float64))
    assert np.all(np.abs(c / kappa - 1) < 1e-2)                    # rounding keeps kappa


@pytest.mark.parametrize("s", [-40, 40])
def test_spd_conditioned_scales_by_a_power_of_two(s):
    a = inputs.spd_conditioned(inputs.rng_for(300, "posv", 16, 3), 3, 16, 1e3, 0)
    b = inputs.spd_conditioned(inputs.rng_for(300, "posv", 16, 3), 3, 16, 1e3, s)
    assert np.array_equal(b, (a.astype(np.float64) * 2.0 ** s).astype(np.float32))   # exact scaling


@pytest.mark.parametrize("kappa", [1e2, 1e4])
@pytest.mark.parametrize("s", [-40, 0, 40])
def test_oracle_on_conditioned_inputs(kappa, s):
    """The FP64 oracle stays far inside the FP32 bars on these inputs:
    factor against LAPACK (numpy), solve against scipy cho_solve, and its
    own residuals at FP64 level."""
    n, b = 48, 6
    case = inputs.make_case("posv", n, b, cfg=300, kappa=kappa, scale_exp=s)
    L, X, info = oracle.posv(case["A"], case["B"])
    assert (info == 0).all()
    A = case["A"].astype(np.float64)
    for p in range(b):
        Lnp = np.linalg.cholesky(A[p])
        assert np.max(np.abs(L[p] - Lnp)) <= 1e-12 * np.max(np.abs(Lnp))
        Xs = sl.cho_solve((Lnp, True), case["B"][p].astype(np.float64))
        assert np.max(np.abs(X[p] - Xs)) <= kappa * 1e-13 * np.max(np.abs(Xs))
        r = np.abs(case["B"][p] - A[p] @ X[p]).max() / (np.abs(A[p]).sum(axis=1).max() * np.abs(X[p]).max())
        assert r <= 1e-14
    Lt = inputs.make_case("trsv", n, b, cfg=300, kappa=kappa, scale_exp=s)
    for trans in (0, 1):
        x = oracle.trsv(Lt["L"], Lt["x"], trans)
        for p in range(b):
            ref = sl.solve_triangular(Lt["L"][p].astype(np.float64), Lt["x"][p].astype(np.float64), lower=True,
                                      trans=trans)
            assert np.max(np.abs(x[p] - ref)) <= 1e-12 * np.max(np.abs(ref)) * np.sqrt(kappa)
