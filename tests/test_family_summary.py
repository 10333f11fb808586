"""The library's family statistics (pa_family_summary, host arithmetic, no
device needed) against the oracle's on the same family arrays, and the
closed forms that pin both."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def B():
    from paper_2006_00561_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("seed", range(4))
def test_matches_the_oracle(B, seed):
    rng = np.random.default_rng(seed)
    n0 = int(rng.integers(1, 2000))
    fam = (rng.zipf(1.4, int(rng.integers(1, 5000))) % n0).astype(np.uint32)
    lib_s = B.family_summary(fam, n0)
    orc = oracle.family_stats(fam, n0)
    assert lib_s["R"] == len(fam) and lib_s["n0"] == n0
    for k in ("families", "largest"):
        assert lib_s[k] == orc[k]
    for k in ("rho_t", "rho_s"):
        assert lib_s[k] == pytest.approx(orc[k], rel=1e-12)


def test_closed_forms_and_errors(B):
    s = B.family_summary(np.arange(100, dtype=np.uint32), 100)
    assert (s["families"], s["largest"], s["rho_t"], s["rho_s"]) == \
        (100, 1, 1.0, 1.0)
    s = B.family_summary(np.full(64, 3, np.uint32), 5)
    assert s["families"] == 1 and s["rho_t"] == pytest.approx(64) and \
        s["rho_s"] == pytest.approx(64)
    with pytest.raises(B.PAError):
        B.family_summary(np.array([0, 5], np.uint32), 5)
    with pytest.raises(B.PAError):
        B.family_summary(np.array([0], np.uint32), 0)
