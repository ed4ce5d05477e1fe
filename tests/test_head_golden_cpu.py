"""The stored oracle doses of the head parity cases are current: written for
the inputs that tests/head_cases.py builds today, by an oracle that computes
the same bits as the one in the tree (fingerprint of a small full-physics
run), at the uncertainty the parity bar needs (U <= 0.3 %), and their stored
voxels reach down to 5 % of the maximum (the comparisons start at 10 %)."""
import numpy as np
import pytest

import head_cases as H


_FP = []


def _fingerprint():
    if not _FP:
        _FP.append(H.oracle_fingerprint())
    return _FP[0]


@pytest.mark.parametrize("name", list(H.CASES))
def test_head_golden_is_current(name):
    c = H.case(name, H.ORACLE_HISTORIES, H.ORACLE_SEED)
    z = np.load(H.golden_file(name), allow_pickle=False)
    assert str(z["input_hash"]) == H.input_hash(c), "regenerate: python tests/golden/make_head_physics.py " + name
    assert str(z["oracle_fingerprint"]) == _fingerprint(), \
        "the oracle computes other bits than when the file was written: python tests/golden/make_head_physics.py"
    assert int(z["n_histories"]) == H.ORACLE_HISTORIES and int(z["seed"]) == H.ORACLE_SEED
    assert int(z["n_batches"]) == H.N_BATCHES
    assert float(z["uncertainty"]) <= 0.003
    d = z["dose_gy"].astype(np.float64)
    assert np.isclose(d.max(), float(z["body_max_gy"]), rtol=1e-6)
    assert d.min() >= H.STORE_FRACTION * d.max() * (1 - 1e-6)
    # batch doses average to the stored dose where both are kept
    pos = np.searchsorted(z["idx"], z["batch_idx"])
    assert np.all(z["idx"][pos] == z["batch_idx"])
    np.testing.assert_allclose(z["batch_dose_gy"].astype(np.float64).mean(axis=0), d[pos], rtol=1e-5)
