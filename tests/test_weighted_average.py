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


def _combined_definition(lnZ, obs, N):
    """The combined observables from their definition in 60-digit
    arithmetic: weights Z_m / sum Z, <E^k> = sum_m w_m sumE^k_m / R_m,
    Var(E) = <E^2> - <E>^2, C = beta^2 Var(E) / N."""
    import mpmath as mp
    mp.mp.dps = 60
    z = [mp.mpf(v) for v in lnZ]
    mx = max(z)
    Z = [mp.e ** (v - mx) for v in z]
    S = sum(Z)
    w = [v / S for v in Z]
    E1 = sum(wi * mp.mpf(o["sumE"]) / o["R"] for wi, o in zip(w, obs))
    E2 = sum(wi * mp.mpf(o["sumE2"]) / o["R"] for wi, o in zip(w, obs))
    A1 = sum(wi * mp.mpf(o["sumAbsM"]) / o["R"] for wi, o in zip(w, obs))
    M2 = sum(wi * mp.mpf(o["sumM2"]) / o["R"] for wi, o in zip(w, obs))
    beta = mp.mpf(obs[0]["beta"])
    var = E2 - E1 * E1
    return {"e": E1 / N, "abs_m": A1 / N, "m2": M2 / (N * N), "varE": var,
            "C": beta * beta * var / N,
            "lnZ": mx + mp.log(S / len(z))}


def _fake_obs(rng, N, R, beta, spread):
    """Integer sums of a population of R energies near -1.6 N (a narrow
    ordered-phase distribution: the variance is a tiny difference of two
    large moments, where a double-precision subtraction loses digits)."""
    E = np.round(-1.6 * N + rng.normal(0, spread, R)).astype(np.int64)
    M = rng.integers(-N, N + 1, R)
    return {"R": R, "beta": beta, "e": 0.0, "abs_m": 0.0, "m2": 0.0,
            "C": 0.0, "sumE": int(E.sum()), "sumE2": int((E * E).sum()),
            "sumAbsM": int(np.abs(M).sum()), "sumM2": int((M * M).sum()),
            "Emin": int(E.min()), "Emax": int(E.max())}


def test_combined_observables_match_the_definition(B):
    rng = np.random.default_rng(3)
    for M, N, R, spread in ((1, 4096, 65536, 40.0), (16, 4096, 20480, 30.0),
                            (48, 256, 1000, 5.0), (5, 16384, 4096, 0.7)):
        beta = 0.4406868
        obs = [_fake_obs(rng, N, R + 17 * m, beta, spread) for m in range(M)]
        lnZ = 3000.0 + rng.normal(0, 0.5, M)
        got = B.combine_observables(lnZ, obs, N)
        ref = _combined_definition(lnZ, obs, N)
        for k in ("e", "abs_m", "m2", "varE", "C", "lnZ"):
            assert abs(got[k] - float(ref[k])) <= 1e-12 * abs(float(ref[k])), k
        assert got["M"] == M and got["R"] == sum(o["R"] for o in obs)


def test_combined_observables_single_population_equals_its_own(B):
    # one population: the combination is that population's own observables
    rng = np.random.default_rng(4)
    N = 1024
    o = _fake_obs(rng, N, 5000, 0.3, 10.0)
    got = B.combine_observables([17.0], [o], N)
    R = o["R"]
    var = (R * o["sumE2"] - o["sumE"] ** 2) / R ** 2   # exact integers
    assert got["e"] == o["sumE"] / R / N
    assert abs(got["varE"] - var) <= 1e-15 * var
    assert got["lnZ"] == 17.0


def test_combined_observables_reject_bad_input(B):
    rng = np.random.default_rng(5)
    a = _fake_obs(rng, 256, 100, 0.3, 3.0)
    b = _fake_obs(rng, 256, 100, 0.31, 3.0)
    with pytest.raises(B.PAError):      # two temperatures
        B.combine_observables([0.0, 0.0], [a, b], 256)
    with pytest.raises(B.PAError):
        B.combine_observables([np.nan], [a], 256)
