"""Weighted averaging over independent populations (pa_weighted_average):
against the definition evaluated in extended precision, and its invariants.
Host arithmetic of the library, no device needed."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def B():
    from paper_2006_00561_amd import binding
    binding.lib()
    return binding


def _definition(lnZ, values):
    """sum_m Z_m O_m / sum_m Z_m and ln((1/M) sum_m Z_m) in long double."""
    z = np.asarray(lnZ, np.longdouble)
    Z = np.exp(z - z.max())
    v = np.asarray(values, np.longdouble)
    avg = (Z[:, None] * v).sum(axis=0) / Z.sum()
    lz = z.max() + np.log(Z.sum() / len(z))
    return avg.astype(np.float64), float(lz)


def test_matches_the_definition(B):
    rng = np.random.default_rng(1)
    for M, k in ((1, 3), (7, 1), (64, 4)):
        lnZ = 1000.0 + rng.normal(0, 3, M)
        vals = rng.normal(0, 10, (M, k))
        out, lz = B.weighted_average(lnZ, vals)
        ref, lref = _definition(lnZ, vals)
        assert np.allclose(out, ref, rtol=1e-13, atol=1e-12)
        assert abs(lz - lref) <= 1e-12 * abs(lref)


def test_invariants(B):
    rng = np.random.default_rng(2)
    vals = rng.normal(0, 1, (5, 2))
    # equal free energies: the plain mean; ln Z unchanged
    out, lz = B.weighted_average(np.full(5, 42.0), vals)
    assert np.allclose(out, vals.mean(axis=0), rtol=1e-15, atol=1e-15)
    assert lz == 42.0
    # one population far ahead dominates
    lnZ = np.array([0.0, 0.0, 60.0, 0.0, 0.0])
    out, lz = B.weighted_average(lnZ, vals)
    assert np.allclose(out, vals[2], rtol=1e-12)
    assert abs(lz - (60.0 - np.log(5.0))) < 1e-12
    # a common shift of ln Z moves only the combined ln Z
    lnZ = rng.normal(0, 2, 5)
    a, la = B.weighted_average(lnZ, vals)
    b, lb = B.weighted_average(lnZ + 123.0, vals)
    assert np.allclose(a, b, rtol=1e-13) and abs(lb - la - 123.0) < 1e-10
    # bad arguments
    with pytest.raises(B.PAError):
        B.weighted_average(np.array([np.inf, 0.0]), vals[:2])
